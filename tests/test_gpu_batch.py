"""GPU: chains run concurrently (worker pool, tempered ladder, serving loop)
give the same results as each chain run alone, and the tempered ladder's
first moves match the FP64 reference."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2511_06407_amd import workloads as wl  # noqa: E402
from oracle import hamiltonian as oham  # noqa: E402
from oracle.chain import run_seeded_chain  # noqa: E402
from tests.parity_util import rel, record, chain_floor  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_06407_amd import rmhmc
    return rmhmc


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def specs_mix():
    a, _ = wl.workload("gp_logistic_d34")
    b, _, _ = wl.gp_logistic_2d(64, seed=5, beta=0.3)
    c, _, _ = wl.propensity_mkl(60, seed=6)
    return [(a, 0.01), (b, 0.01), (dataclasses.replace(c, jitter=1e-2), 0.003)]


def test_pool_mix_equals_alone(rm):
    n_moves, C_, K = 3, 2, 6
    runs = []
    for k, (spec, eps) in enumerate(specs_mix()):
        runs.append((spec, eps, dev(np.zeros(spec.D)), k))
    alone = []
    for spec, eps, q0, k in runs:
        s, l, a, st = rm.Model(spec).chain(q0, eps, C_, K, n_moves, seed=1, stream_id=k)
        torch.cuda.synchronize()
        alone.append((s.cpu().numpy(), l.cpu().numpy(), a.cpu().numpy()))
    pool = rm.Pool(3)
    models = [rm.Model(spec) for spec, *_ in runs]
    jobs = [pool.submit(m, q0, eps, C_, K, n_moves, seed=1, stream_id=k)
            for m, (spec, eps, q0, k) in zip(models, runs)]
    for j in jobs:
        assert pool.wait(j)
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        s, l, a = j.samples.cpu().numpy(), j.logpost.cpu().numpy(), j.accepted.cpu().numpy()
        record("pool_mix", chain=k, D=runs[k][0].D, samples=rel(s, alone[k][0]),
               accepted=int(a.sum()), start_ms=j.times_ms[1], end_ms=j.times_ms[2])
        assert np.array_equal(s, alone[k][0]) and np.array_equal(l, alone[k][1])
        assert np.array_equal(a, alone[k][2])
    # the jobs overlapped in time
    starts = [j.times_ms[1] for j in jobs]
    ends = [j.times_ms[2] for j in jobs]
    assert max(starts) < min(ends)
    pool.close()


def test_tempered_ladder_runs_and_matches_reference(rm):
    from paper_2511_06407_amd.tempered import run_tempered
    out = run_tempered(n_chains=6, n_moves=2, n_leapfrog=2, n_workers=3, seed=0, engine="pool")
    record("tempered", wall_s=out["wall_s"], leapfrogs=out["chain_leapfrogs"],
           lf_per_s=out["chain_leapfrogs_per_s"])
    assert out["chain_leapfrogs"] > 0
    # reference for the smallest chain
    k = int(np.argmin([c["D"] for c in out["chains"]]))
    specs, dims, betas = wl.tempered_ladder(6, 0)
    spec = specs[k]
    ref = run_seeded_chain(oham.GPTarget(spec), np.zeros(spec.D), 0.01, 2, 6, 1e6, 2, 0, 0, k)
    got = out["jobs"][k].samples.cpu().numpy()
    e = rel(got, ref[0])
    fl = chain_floor(spec, 0.01, 2, 6, 1e6, 2, 0, k, ref)
    bar = max(1e-10, 10 * fl)
    record("tempered_ref", chain=k, D=spec.D, beta=float(betas[k]), samples=e, floor=fl, bar=bar)
    assert np.array_equal(out["jobs"][k].accepted.cpu().numpy(), ref[2])
    assert e < bar


def test_serving_results_same_alone_and_in_mix(rm):
    from paper_2511_06407_amd import serving as sv
    reqs = sv.make_requests(8.0, 0.6, d_min=34, d_max=140, moves=(2, 3), seed=3)
    assert len(reqs) >= 3
    ex = sv.PoolExecutor(n_workers=3, n_leapfrog=2)
    kept = {}
    start = ex.start

    def start_keep(r):
        j = start(r)
        kept[r.rid] = j
        return j
    ex.start = start_keep
    sch = sv.Scheduler(ex, hbm_budget_bytes=60e9, n_slots=3)
    sch.run(reqs)
    summ = sv.summarize(reqs, max(r.done_s for r in reqs))
    record("serving", **{k: v for k, v in summ.items()})
    assert sch.max_running >= 2
    for r in reqs[:3]:
        spec, eps = sv.request_spec(r)
        s, l, a, st = rm.Model(spec).chain(dev(np.zeros(spec.D)), eps, 2, 6, r.n_moves,
                                           seed=r.seed, stream_id=r.rid)
        torch.cuda.synchronize()
        assert np.array_equal(s.cpu().numpy(), kept[r.rid].samples.cpu().numpy())
    ex.close()


def test_serving_largest_requests_same_alone_and_in_pool(rm):
    """The serving mix's largest requests (D = 1038, both model kinds) run
    side by side on the pool: every workspace at its largest size, and each
    result bitwise that of the same request alone."""
    from paper_2511_06407_amd import serving as sv
    reqs = [sv.Request(0, 0.0, "gp_logistic", 1038, 1, seed=11),
            sv.Request(1, 0.0, "mkl", 1038, 1, seed=12)]
    C_, K = 2, 6
    runs = []
    for r in reqs:
        spec, eps = sv.request_spec(r)
        runs.append((spec, eps, dev(np.zeros(spec.D)), r))
    alone = []
    for spec, eps, q0, r in runs:
        s, l, a, st = rm.Model(spec).chain(q0, eps, C_, K, r.n_moves, seed=r.seed,
                                           stream_id=r.rid)
        torch.cuda.synchronize()
        alone.append((s.cpu().numpy(), l.cpu().numpy(), a.cpu().numpy()))
    pool = rm.Pool(2)
    models = [rm.Model(spec) for spec, *_ in runs]
    jobs = [pool.submit(m, q0, eps, C_, K, r.n_moves, seed=r.seed, stream_id=r.rid)
            for m, (spec, eps, q0, r) in zip(models, runs)]
    for j in jobs:
        assert pool.wait(j)
    torch.cuda.synchronize()
    for k, j in enumerate(jobs):
        s, l, a = j.samples.cpu().numpy(), j.logpost.cpu().numpy(), j.accepted.cpu().numpy()
        record("serving_largest", kind=reqs[k].kind, D=runs[k][0].D, samples=rel(s, alone[k][0]),
               accepted=int(a.sum()))
        assert np.all(np.isfinite(s))
        assert np.array_equal(s, alone[k][0]) and np.array_equal(l, alone[k][1])
        assert np.array_equal(a, alone[k][2])
    pool.close()


def test_graph_batch_equals_eager_chain_and_alone(rm):
    """Chains whose moves are replayed from captured graphs: identical to
    themselves admitted alone, and to the eager rmhmc_chain on the same model
    with the same (tuned) launch shapes."""
    n_moves, C_, K = 3, 2, 6
    runs = []
    for k, (spec, eps) in enumerate(specs_mix()):
        runs.append((spec, eps, dev(np.zeros(spec.D)), k))
    models = [rm.Model(spec) for spec, *_ in runs]
    # alone: one chain per batch (admission tunes the chain's class and sets
    # the model's launch shapes; later runs reuse them)
    alone = []
    for m, (spec, eps, q0, k) in zip(models, runs):
        b = rm.Batch(1)
        j = b.admit(m, q0, eps, C_, K, n_moves, seed=4, stream_id=k)
        b.step(n_moves)
        b.sync()
        b.retire(j)
        b.close()
        alone.append((j.samples.cpu().numpy(), j.logpost.cpu().numpy(), j.accepted.cpu().numpy(),
                      j.stats, j.shape))
    # the eager chain on the same models (now with the tuned launch shapes)
    eager = []
    for m, (spec, eps, q0, k) in zip(models, runs):
        s, l, a, st = m.chain(q0, eps, C_, K, n_moves, seed=4, stream_id=k)
        torch.cuda.synchronize()
        eager.append((s.cpu().numpy(), l.cpu().numpy(), a.cpu().numpy()))
    # mixed: all chains in one batch on two streams
    b = rm.Batch(2)
    jobs = [b.admit(m, q0, eps, C_, K, n_moves, seed=4, stream_id=k)
            for m, (spec, eps, q0, k) in zip(models, runs)]
    b.step(n_moves)
    b.sync()
    for k, j in enumerate(jobs):
        b.retire(j)
        s, l, a = j.samples.cpu().numpy(), j.logpost.cpu().numpy(), j.accepted.cpu().numpy()
        record("graph_batch", chain=k, D=runs[k][0].D, moves=j.moves_done,
               accepted=int(a.sum()), sweep_budget=j.shape["sweep_budget"],
               gsplit=j.shape["gsplit"], noconv=j.stats.fail_noconv,
               vs_eager=rel(s, eager[k][0]))
        assert j.moves_done == n_moves and j.stats.leapfrogs == n_moves * C_
        assert j.stats.fail_noconv == 0
        assert np.array_equal(s, alone[k][0]) and np.array_equal(l, alone[k][1])
        assert np.array_equal(a, alone[k][2])
        assert np.array_equal(s, eager[k][0]) and np.array_equal(a, eager[k][2])
    b.close()
    # a model in a batch is refused elsewhere until retired
    b = rm.Batch(1)
    j = b.admit(models[0], runs[0][2], runs[0][1], C_, K, n_moves, seed=4)
    with pytest.raises(rm.RmhmcError):
        models[0].chain(runs[0][2], runs[0][1], C_, K, n_moves)
    b.step(n_moves)
    b.retire(j)
    b.close()


def test_graph_tempered_ladder_matches_reference(rm):
    """The tempered ladder on the graph engine: the smallest chain's first
    moves against the reference chain within 10 x its permutation floor."""
    from paper_2511_06407_amd.tempered import run_tempered
    out = run_tempered(n_chains=6, n_moves=2, n_leapfrog=2, n_workers=3, seed=0, engine="graph")
    record("tempered_graph", wall_s=out["wall_s"], setup_s=out["setup_s"],
           leapfrogs=out["chain_leapfrogs"], lf_per_s=out["chain_leapfrogs_per_s"])
    k = int(np.argmin([c["D"] for c in out["chains"]]))
    specs, dims, betas = wl.tempered_ladder(6, 0)
    spec = specs[k]
    ref = run_seeded_chain(oham.GPTarget(spec), np.zeros(spec.D), 0.01, 2, 6, 1e6, 2, 0, 0, k)
    got = out["jobs"][k].samples.cpu().numpy()
    fl = chain_floor(spec, 0.01, 2, 6, 1e6, 2, 0, k, ref)
    bar = max(1e-10, 10 * fl)
    e = rel(got, ref[0])
    record("tempered_graph_ref", chain=k, D=spec.D, samples=e, floor=fl, bar=bar)
    assert np.array_equal(out["jobs"][k].accepted.cpu().numpy(), ref[2])
    assert e < bar
