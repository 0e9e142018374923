"""Benchmark: exponential-shift low-diameter decomposition on one MI355X.

One step = one whole decomposition (Delta reduction, wake-round sort, all rounds, centre
extraction, cut count) of the RMAT scale-24 graph (edge factor 16, a,b,c = .57,.19,.19,
symmetrised, relabelled; 16.7M vertices, 260M edges) with beta = 0.05 and seeded Exp
shifts, inputs resident in HBM.  Prints one JSON line.

  value        GTEPS = undirected edges / seconds per step (whole graph)
  roofline     the round kernel: algorithmic bytes per launch over its average launch
               duration (HIP events on the launch stream), against 8 TB/s HBM3E; traffic from
               the committed rocprofv3 counter runs when they match the current kernel sources
  batched      512 uneven graphs in one call (workgroup engine: one workgroup, or a team of
               workgroups for the largest graphs, per graph) vs one call each
  served       a Poisson stream of RMAT 12-22 requests through the serving engine vs the same
               stream one decomposition at a time (FIFO), latency p50 / p99 and capacity
  grid2d       grid 64x64: p50 / p99 latency over 1000 calls
  grid3d       grid 256^3 with the tuner's engine and mapping: time, round steps, the round
               kernel's roofline (and the untuned time)
  shift_variants  Sec. 5's permutation variants of the shifts vs Exp shifts: cut and radius
  cpu_baseline the CPU oracle's bucketed search (single-threaded, one core) on the same graph and shifts

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat-24]
                       [--engine E] [--blocks B] [--direction D] [--tail-vertices T]
                       [--no-batch] [--no-serve] [--no-grids] [--no-cpu-baseline] [--copy-probe]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS + decompositions/s, p50/p99 latency; batched vs plain, bit-exact"
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_rounds.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(st, n):
    """Bytes the round kernel must move over one decomposition:
    per arc examined, its column id (4 B) and the far end's label (8 B);
    per vertex with arcs, its wake-order entry (4 B) and shift (8 B) when woken, its two row
    offsets (8 B), its label written (8 B), and its queue entry (vertex and arc prefix, 8 B)
    written and read back (16 B): 44 B;
    per pull pass (every bottom-up round and the tail seed), every label read once (8 B)."""
    pulls = st["bu_rounds"] + (1 if st["tail_round"] >= 0 else 0)
    return 12 * st["arcs_examined"] + 44 * st["n_active"] + 8 * n * pulls


def kernel_sources_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1307_3692_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter runs
    (profiles/traffic_rounds.json: one entry per workload and kernel), or None when they were
    taken on other kernel sources, another workload or another kernel."""
    if not os.path.exists(TRAFFIC):
        return None
    with open(TRAFFIC) as f:
        t = json.load(f)
    sha = kernel_sources_sha()
    for e in t.get("entries", []):
        if e.get("workload") == workload and e.get("kernel") == kernel and e.get("kernel_sources_sha") == sha:
            return e.get("bytes_per_launch")
    return None


def sha_array(a):
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def pack(graphs):
    import numpy as np
    vo, ao = [0], [0]
    for rp, ci, s, _ in graphs:
        vo.append(vo[-1] + rp.size - 1)
        ao.append(ao[-1] + ci.size)
    return (vo, ao, np.concatenate([g[0] for g in graphs]), np.concatenate([g[1] for g in graphs]),
            np.concatenate([g[2] for g in graphs]))


def run_batched(reps: int, plain_reps: int = 1):
    """The batched workload (512 ER / random-geometric graphs, 1k-200k vertices each, own beta
    and seeds): one ldd_decompose_batch call (the workgroup engine: one workgroup runs all rounds
    of a graph, largest graphs first) against the plain path (one ldd_decompose per graph), same
    inputs, same bits; the disjoint-union engine (one launch per round step for all graphs) is
    timed beside them."""
    import numpy as np
    import torch

    import inputs
    import paper_1307_3692_amd as ldd

    t = time.time()
    graphs = inputs.batch_graphs(512, seed=1)
    vo, ao, rp, ci, s = pack(graphs)
    m = ao[-1] // 2
    log(f"batch-512: {vo[-1]} vertices, {m} edges, generated in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    d_rp, d_ci, d_s = (torch.from_numpy(a).to(dev) for a in (rp, ci, s))
    centre = torch.empty(vo[-1], dtype=torch.int32, device=dev)
    ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, centre=centre)  # warm-up
    torch.cuda.synchronize()
    # the engine's mapping for this batch, from the library's tuner (outside the timed runs)
    t = time.time()
    tuned, tune_rep = ldd.tune(d_rp, d_ci, d_s, vtx_off=vo, arc_off=ao, centre=centre)
    log(f"batch-512: tuned {tuned} {tune_rep} in {time.time() - t:.1f}s")
    lat = []
    for _ in range(reps):
        a = time.perf_counter()
        _, cuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, centre=centre, **tuned)
        lat.append(time.perf_counter() - a)
    union_centre = centre.cpu().numpy()
    # the same batch on the disjoint-union engine (one launch per round step for all graphs)
    uni = []
    for _ in range(reps):
        a = time.perf_counter()
        _, ucuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, centre=centre, batch_mode=ldd.BATCH_UNION)
        uni.append(time.perf_counter() - a)
    same_union = bool(np.array_equal(union_centre, centre.cpu().numpy()) and cuts == ucuts)
    plain = []
    for _ in range(plain_reps):
        a = time.perf_counter()
        _, pcuts = ldd.decompose_batch(vo, ao, d_rp, d_ci, d_s, centre=centre, batch_mode=ldd.BATCH_SEQUENTIAL)
        plain.append(time.perf_counter() - a)
    same = bool(np.array_equal(union_centre, centre.cpu().numpy()) and cuts == pcuts)
    bit_exact = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            gold = json.load(f).get("batch-512")
        if gold:
            bit_exact = bool(hashlib.sha256(union_centre.view(np.uint8)).hexdigest() == gold["sha_centre"]
                             and hashlib.sha256(np.array(cuts, np.int64).view(np.uint8)).hexdigest()
                             == gold["sha_cuts"])
    t_union, t_plain = float(np.median(lat)), float(np.median(plain))
    out = {"workload": "batch-512: 512 graphs, n log-uniform 1k-200k, half Erdos-Renyi mean degree 8, half 2D "
                       "random geometric mean degree 6, beta log-uniform [0.02, 0.3], seed 1",
           "n": vo[-1], "m": m, "reps": reps,
           "decompositions_per_s": round(512 / t_union, 1),
           "gteps": round(m / t_union / 1e9, 3),
           "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
           "plain_decompositions_per_s": round(512 / t_plain, 1),
           "plain_ms": round(t_plain * 1e3, 3),
           "speedup_vs_plain": round(t_plain / t_union, 2),
           "engine": "workgroup (one workgroup per graph, or a team of workgroups for the largest; "
                     "the heaviest per workgroup first)",
           "union_engine_ms": round(float(np.median(uni)) * 1e3, 3), "union_identical": same_union,
           "tuned": tuned,
           "untuned_ms": round(tune_rep["default_ms"], 3), "tuned_ms": round(tune_rep["best_ms"], 3),
           "identical_to_plain": same, "bit_exact": bit_exact}
    log(f"batched: {out}")
    return out


def serve_templates(dev):
    """The request pool: RMAT scale 12..22 (edge factor 16, graph seed 1000 + scale), each with
    beta in {0.05, 0.1, 0.2} and two shift seeds: 66 distinct (graph, beta, shifts) templates,
    device-resident (inputs.serve_recipe).  A request stream draws templates uniformly, so its
    scale is uniform in 12..22 and its beta uniform in the three values."""
    import torch

    import inputs
    out, graphs = [], {}
    for scale, beta, gseed, sseed in inputs.serve_recipe():
        if scale not in graphs:
            rp, ci = inputs.rmat(scale, 16, seed=gseed)
            graphs = {scale: (torch.from_numpy(rp).to(dev), torch.from_numpy(ci).to(dev), rp.size - 1, ci.size // 2)}
        d_rp, d_ci, n, m = graphs[scale]
        d_s = torch.from_numpy(inputs.make_shifts(n, beta, sseed)).to(dev)
        out.append({"scale": scale, "beta": beta, "seed": sseed, "n": n, "m": m, "rp": d_rp, "ci": d_ci, "s": d_s})
    return out


def fifo_latencies(arrivals, service):
    """One worker, first come first served: latency of each request (same unit as inputs)."""
    import numpy as np
    done = np.empty_like(arrivals)
    t = -np.inf
    for i, (a, s) in enumerate(zip(arrivals, service)):
        t = max(t, a) + s
        done[i] = t
    return done - arrivals


def plain_run(ldd, tm, req, arrivals, bufs):
    """The plain path under the same kind of load: one ldd_decompose per request in arrival order,
    each started no earlier than its arrival (offsets in seconds); latency (ms) from the arrival
    to the call's return (the call returns with its cut on the host)."""
    import numpy as np
    lat = np.zeros(len(req))
    t0 = time.perf_counter()
    for i, ti in enumerate(req):
        due = t0 + arrivals[i]
        while True:
            now = time.perf_counter()
            if now >= due:
                break
            if due - now > 2e-3:
                time.sleep(due - now - 1e-3)
        x = tm[ti]
        ldd.decompose(x["rp"], x["ci"], x["s"], x["beta"], centre=bufs[ti])
        lat[i] = time.perf_counter() - due
    return lat * 1e3


def serve_run(ldd, srv, tm, req, outs, arrivals=None):
    """Submit requests (all at once, or at the given arrival offsets in seconds), collect them
    on a second thread; returns per-request latency (ms) and the run's wall span (s)."""
    import threading

    import numpy as np
    N = len(req)
    tickets = [None] * N
    sub_py = np.zeros(N)
    lag = np.zeros(N)
    results = [None] * N
    ready = [threading.Event() for _ in range(N)]

    def collect():
        for i in range(N):
            ready[i].wait()
            results[i] = srv.wait(tickets[i])

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    for i, t in enumerate(req):
        if arrivals is not None:
            due = t0 + arrivals[i]
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                if due - now > 2e-3:
                    time.sleep(due - now - 1e-3)
        sub_py[i] = time.perf_counter()
        lag[i] = sub_py[i] - (t0 + arrivals[i]) if arrivals is not None else 0.0
        tickets[i] = srv.submit(tm[t]["rp"], tm[t]["ci"], tm[t]["s"], centre=outs[i])
        ready[i].set()
    th.join()
    lat = np.array([r[2]["latency_ms"] for r in results]) + lag * 1e3
    done_py = sub_py + np.array([(r[2]["t_done"] - r[2]["t_submit"]) for r in results])
    start = t0 if arrivals is not None else sub_py[0]
    return lat, float(done_py.max() - start), results


def run_serving(n_requests: int = 2000, budget_gib: float = 16.0, small_budget_gib: float = 0.25):
    """Serving: a stream of RMAT 12-22 requests through ldd_server_* (continuous batching into
    one device-resident arena) against the plain path (one ldd_decompose per request, FIFO).
    Capacity comes from a saturating closed loop; latency from Poisson arrivals at 80% of it.
    The plain path's latency at its own 80% load is a real run of the same arrival pattern
    (scaled to its capacity); the FIFO model over its measured service times is kept beside it,
    and also gives the plain latency at the server's arrival rate, which plain cannot sustain."""
    import numpy as np
    import torch

    import paper_1307_3692_amd as ldd
    dev = torch.device("cuda:0")
    t = time.time()
    tm = serve_templates(dev)
    log(f"serve: {len(tm)} templates generated in {time.time() - t:.1f}s")
    rng = np.random.default_rng(1)
    req = rng.integers(0, len(tm), n_requests)
    # reference results: the plain path's result of each template, checked against the oracle's
    # digest of that template; every served request is then compared with it on the device
    gold = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            gold = json.load(f).get("serve-templates", {}).get("templates")
    ref, ref_oracle = [], []
    for i, x in enumerate(tm):
        c, cut = ldd.decompose(x["rp"], x["ci"], x["s"], x["beta"])
        ref.append((c, cut))
        if gold:
            ref_oracle.append(sha_array(c.cpu().numpy()) == gold[i]["sha_centre"] and cut == gold[i]["cut"])
    templates_vs_oracle = bool(gold) and all(ref_oracle)
    # plain: the request stream one ldd_decompose at a time
    service = np.zeros(n_requests)
    plain_out = {}
    for i, ti in enumerate(req):
        x = tm[ti]
        buf = plain_out.setdefault(ti, torch.empty(x["n"], dtype=torch.int32, device=dev))
        a = time.perf_counter()
        ldd.decompose(x["rp"], x["ci"], x["s"], x["beta"], centre=buf)
        service[i] = time.perf_counter() - a
    plain_cap = n_requests / service.sum()
    log(f"serve: plain {plain_cap:.1f} req/s, mean {service.mean() * 1e3:.3f} ms")
    outs = [torch.empty(tm[ti]["n"], dtype=torch.int32, device=dev) for ti in req]
    torch.cuda.synchronize()

    def verify(results):
        ok = True
        for i, ti in enumerate(req):
            c, cut, _ = results[i]
            ok &= bool(torch.equal(c, ref[ti][0])) and cut == ref[ti][1]
        return ok

    out = {"workload": f"serving: {n_requests} requests, RMAT scale uniform 12-22 (edge factor 16, graph seed "
                       "1000+scale), beta uniform in {0.05, 0.1, 0.2}, shift seeds 1000+6(scale-12)+2j+k "
                       "(66 device-resident templates), template stream seed 1",
           "requests": n_requests, "mean_edges": round(float(np.mean([tm[i]["m"] for i in req])), 1)}
    with ldd.Server(hbm_budget_bytes=int(budget_gib * 2**30)) as srv:
        serve_run(ldd, srv, tm, req[:64], outs[:64])  # warm-up
        lat_c, span_c, res_c = serve_run(ldd, srv, tm, req, outs)
        cap = n_requests / span_c
        same_c = verify(res_c)
        lam = 0.8 * cap
        arr = np.cumsum(np.random.default_rng(2).exponential(1.0 / lam, n_requests))
        lat_p, span_p, res_p = serve_run(ldd, srv, tm, req, outs, arrivals=arr)
        same_p = verify(res_p)
        info = srv.info()
    log(f"serve: capacity {cap:.1f} req/s, poisson p50 {np.percentile(lat_p, 50):.3f} ms, info {info}")
    plain_same = fifo_latencies(arr, service) * 1e3
    arr_own = arr * (lam / (0.8 * plain_cap))
    plain_own = fifo_latencies(arr_own, service) * 1e3
    plain_own_run = plain_run(ldd, tm, req, arr_own, plain_out)
    out.update({
        "hbm_budget_gib": budget_gib, "arena_vertices": info["arena_vertices"], "arena_arcs": info["arena_arcs"],
        "capacity_req_per_s": round(cap, 1),
        "closed_loop_p50_ms": round(float(np.percentile(lat_c, 50)), 3),
        "poisson_lambda_req_per_s": round(lam, 1),
        "poisson_throughput_req_per_s": round(n_requests / span_p, 1),
        "poisson_gteps": round(float(sum(tm[i]["m"] for i in req)) / span_p / 1e9, 3),
        "p50_ms": round(float(np.percentile(lat_p, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_p, 99)), 3),
        "max_active": info["max_active"], "rebases": info["rebases"],
        "plain_capacity_req_per_s": round(plain_cap, 1),
        "plain_mean_service_ms": round(float(service.mean()) * 1e3, 4),
        "plain_at_same_lambda_p50_ms": round(float(np.percentile(plain_same, 50)), 3),
        "plain_at_same_lambda_p99_ms": round(float(np.percentile(plain_same, 99)), 3),
        "plain_at_own_80pct_p50_ms": round(float(np.percentile(plain_own_run, 50)), 3),
        "plain_at_own_80pct_p99_ms": round(float(np.percentile(plain_own_run, 99)), 3),
        "plain_at_own_80pct_model_p50_ms": round(float(np.percentile(plain_own, 50)), 3),
        "plain_at_own_80pct_model_p99_ms": round(float(np.percentile(plain_own, 99)), 3),
        "speedup_capacity_vs_plain": round(cap / plain_cap, 2),
        "identical_to_plain": bool(same_c and same_p),
        "bit_exact": bool(same_c and same_p and templates_vs_oracle),
    })
    if small_budget_gib:
        with ldd.Server(hbm_budget_bytes=int(small_budget_gib * 2**30)) as srv:
            lat_s, span_s, res_s = serve_run(ldd, srv, tm, req, outs)
            info_s = srv.info()
        out["small_budget"] = {"hbm_budget_gib": small_budget_gib, "arena_vertices": info_s["arena_vertices"],
                               "arena_arcs": info_s["arena_arcs"],
                               "capacity_req_per_s": round(n_requests / span_s, 1),
                               "closed_loop_p50_ms": round(float(np.percentile(lat_s, 50)), 3),
                               "closed_loop_p99_ms": round(float(np.percentile(lat_s, 99)), 3),
                               "max_active": info_s["max_active"], "identical_to_plain": verify(res_s)}
    log(f"served: {out}")
    return out


def golden(name):
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        return json.load(f).get(name)


def round_kernel(stats, engine):
    """The dominant kernel of a decomposition: the workgroup engines (one step, no frontier
    statistics, also when the automatic choice took them) run everything in k_block_decompose."""
    if engine in (3, 4) or (stats["steps"] == 1 and stats["max_frontier"] == 0):
        return "k_block_decompose"
    return "k_rounds_persistent" if engine == 1 else "k_round_step_lb"


def roofline_block(stats, n, kernel, traffic=None):
    """The round kernel's algorithmic bytes per launch over its average launch duration (HIP
    events around the launches on their stream, idle launches included)."""
    t_rounds = stats["ms_rounds"] * 1e-3
    launches = max(1, stats["steps"])
    alg = algorithmic_bytes(stats, n)
    achieved = (alg / launches) / (t_rounds / launches) / 1e9 if t_rounds > 0 else 0.0
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(alg / launches), "launches": launches,
            "avg_launch_us": round(t_rounds / launches * 1e6, 3)}


def run_single(ldd, name, steps, warmup, opts, keep_host=False, tune=False):
    """Decompose one named workload `steps` times after `warmup` untimed calls, inputs resident
    in HBM; per-call latency from the host clock; stage times and counters from the library, taken
    by up to five further calls with statistics (whose extra pass, the largest distance to a
    centre, is not part of the timed calls).
    With `tune`, the library's tuner picks the engine and its mapping first (outside the timed
    calls) and the timed calls use its choice."""
    import numpy as np
    import torch

    import inputs
    t = time.time()
    rp, ci, s, beta = inputs.workload(name)
    n, m = rp.size - 1, ci.size // 2
    log(f"workload {name}: n={n} m={m} beta={beta} generated in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    d_rp, d_ci, d_s = (torch.from_numpy(a).to(dev) for a in (rp, ci, s))
    centre = torch.empty(n, dtype=torch.int32, device=dev)
    for _ in range(warmup):
        ldd.decompose(d_rp, d_ci, d_s, beta, centre=centre, **opts)
    torch.cuda.synchronize()
    tuned = None
    if tune:
        t = time.time()
        opts, tuned = ldd.tune(d_rp, d_ci, d_s, centre=centre, **opts)
        log(f"workload {name}: tuned {opts} {tuned} in {time.time() - t:.1f}s")
    # the timed calls: the decomposition alone (centres and cut; no statistics pass)
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        _, cut = ldd.decompose(d_rp, d_ci, d_s, beta, centre=centre, **opts)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    gold = golden(name)
    bit_exact = None
    if gold:
        bit_exact = bool(sha_array(centre.cpu().numpy()) == gold["sha_centre"] and cut == gold["cut"])
    # counters and per-stage device times (HIP events) from further calls with statistics
    stage = [ldd.decompose(d_rp, d_ci, d_s, beta, centre=centre, stats=True, **opts)[2] for _ in range(min(steps, 5))]
    # medians of the per-call device times (HIP events)
    med = {k: float(np.median([st[k] for st in stage])) for k in ("ms_prep", "ms_rounds", "ms_finalize", "ms_cut")}
    stats = dict(stage[-1])
    stats.update(med)
    out = {"name": name, "n": n, "m": m, "beta": beta, "lat": lat, "ms_per_step": total / steps * 1e3,
           "stats": stats, "bit_exact": bit_exact, "cut": cut, "opts": opts, "tune_report": tuned}
    if keep_host:
        out["host"] = (rp, ci, s)
    del d_rp, d_ci, d_s, centre
    torch.cuda.empty_cache()
    return out


def run_grid2d(ldd, calls=1000):
    """The small high-overhead case: grid 64x64, beta 0.1, shift seed 1; latency of each of
    `calls` decompositions (host clock around the call, which returns with the cut on the host)."""
    import numpy as np
    r = run_single(ldd, "grid2d-64x64", calls, 20, {})
    lat = np.array(r["lat"]) * 1e3
    st = r["stats"]
    out = {"workload": "grid2d-64x64: 4-neighbour grid 64x64 (4096 vertices, 8064 edges), beta 0.1, shift seed 1",
           "calls": calls, "p50_ms": round(float(np.percentile(lat, 50)), 4),
           "p99_ms": round(float(np.percentile(lat, 99)), 4), "mean_ms": round(float(lat.mean()), 4),
           "decompositions_per_s": round(1e3 / float(lat.mean()), 1),
           "rounds": st["rounds"], "steps": st["steps"], "tail_sweeps": st["tail_iters"],
           "bit_exact": r["bit_exact"]}
    log(f"grid2d: {out}")
    return out


def run_grid3d(ldd, steps=5):
    """The high-diameter case: grid 256^3, beta 0.02, shift seed 1: time per decomposition, round
    steps and the round kernel's roofline."""
    import numpy as np
    r = run_single(ldd, "grid3d-256", steps, 2, {}, tune=True)
    st = r["stats"]
    ms = float(np.median(r["lat"])) * 1e3
    rep = r["tune_report"]
    out = {"workload": "grid3d-256: 6-neighbour grid 256^3 (16.7M vertices, 50.1M edges), beta 0.02, shift seed 1",
           "ms": round(ms, 3), "ms_per_step": round(r["ms_per_step"], 3),
           "gteps": round(r["m"] / (ms * 1e-3) / 1e9, 3),
           "rounds": st["rounds"], "rounds_bound": st["rounds_bound"], "tail_sweeps": st["tail_iters"],
           "steps": st["steps"], "us_per_step": round(st["ms_rounds"] * 1e3 / max(1, st["steps"]), 2),
           "arcs_examined": st["arcs_examined"],
           "stage_ms": {k: round(st[k], 4) for k in ("ms_prep", "ms_rounds", "ms_finalize", "ms_cut")},
           "roofline": roofline_block(st, r["n"], round_kernel(st, r["opts"].get("engine", 0)),
                                      measured_traffic("grid3d-256", round_kernel(st, r["opts"].get("engine", 0)))),
           "tuned": r["opts"], "untuned_ms": round(rep["default_ms"], 3), "tuned_ms": round(rep["best_ms"], 3),
           "bit_exact": r["bit_exact"]}
    log(f"grid3d: {out}")
    return out


def run_shift_variants(ldd, seeds=10):
    """Sec. 5's closing remarks: integer shifts with a random-ranking tie-break, and shifts taken
    from positions in a random ranking, against the Exp(beta) shifts -- the cut fraction and the
    largest distance to a centre over seeded draws, each decomposition by the library."""
    import numpy as np
    import torch

    import inputs
    dev = torch.device("cuda:0")
    names = {ldd.SHIFTS_EXP: "exp", ldd.SHIFTS_INT_PERM: "integer+ranking", ldd.SHIFTS_PERM_ORDER: "ranking positions"}
    out = []
    for gname, (rp, ci), beta in (("grid2d-1000", inputs.grid2d(1000, 1000), 0.01),
                                  ("grid2d-1000", inputs.grid2d(1000, 1000), 0.05),
                                  ("rmat-20", inputs.rmat(20, 16, seed=1), 0.2)):
        n, m = rp.size - 1, ci.size // 2
        d_rp, d_ci = torch.from_numpy(rp).to(dev), torch.from_numpy(ci).to(dev)
        centre = torch.empty(n, dtype=torch.int32, device=dev)
        for kind, kname in names.items():
            cuts, radii, pieces = [], [], []
            for sd in range(seeds):
                s = torch.from_numpy(ldd.make_shifts_variant(n, beta, 100 + sd, kind)).to(dev)
                _, cut, st = ldd.decompose(d_rp, d_ci, s, beta, centre=centre, stats=True)
                cuts.append(cut / m)
                radii.append(st["max_radius"])
                pieces.append(st["pieces"])
            out.append({"graph": gname, "beta": beta, "shifts": kname, "draws": seeds,
                        "cut_fraction_mean": round(float(np.mean(cuts)), 6), "cut_fraction_sd": round(float(np.std(cuts)), 6),
                        "max_radius_mean": round(float(np.mean(radii)), 2), "max_radius_sd": round(float(np.std(radii)), 2),
                        "pieces_mean": round(float(np.mean(pieces)), 1)})
            log(f"shift variants: {out[-1]}")
    return out


def cpu_host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


CPU_CHILD = r"""
import os, sys, time, json
sys.path.insert(0, sys.argv[1])
os.sched_setaffinity(0, {int(sys.argv[3])})
import numpy as np
import inputs, oracle
rp, ci, s, beta = inputs.workload(sys.argv[2])
times = []
for _ in range(int(sys.argv[4])):
    t = time.perf_counter()
    oracle.decompose_rounds(rp, ci, s)
    times.append(time.perf_counter() - t)
print(json.dumps({"times": times, "m": int(ci.size // 2), "n": int(rp.size - 1)}))
"""


def cpu_baseline(name, runs=3):
    """The CPU oracle's bucketed search (one integer distance per round, single-threaded) on the
    same graph and shifts as the GPU run, in a child process pinned to one core: median of
    `runs` runs, generation excluded."""
    import subprocess
    model, ncpu, avail = cpu_host_info()
    core = sorted(os.sched_getaffinity(0))[-1]
    p = subprocess.run([sys.executable, "-c", CPU_CHILD, ROOT, name, str(core), str(runs)], capture_output=True,
                       text=True, check=True)
    r = json.loads(p.stdout.strip().splitlines()[-1])
    times = sorted(r["times"])
    med = times[len(times) // 2]
    return {"value": round(r["m"] / med / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{name}: the whole benchmark graph and shifts (n={r['n']}, m={r['m']}), bucketed search "
                      f"(oracle.decompose_rounds), median of {runs} runs ({', '.join(f'{t:.2f}' for t in r['times'])} s) "
                      f"on one core (pinned to cpu {core}) of this host",
            "cpu_model": model, "nproc": ncpu, "cpus_available": avail}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat-24")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-grids", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the steps, copy 1 GiB three times (a plain copy kernel of known size, to "
                         "calibrate HBM byte counters taken in the same run)")
    ap.add_argument("--engine", type=int, default=0)
    ap.add_argument("--direction", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--tail-vertices", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the decomposition of one graph "
              "is sized for one MI355X and the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1307_3692_amd as ldd

    opts = dict(engine=args.engine, direction=args.direction, blocks=args.blocks, tail_vertices=args.tail_vertices)
    r = run_single(ldd, args.workload, args.steps, args.warmup, opts)
    stats, n, m = r["stats"], r["n"], r["m"]
    ms_step = r["ms_per_step"]
    log(f"steps {args.steps}: {ms_step:.3f} ms/step, stats {stats}")
    if args.copy_probe:
        dev = torch.device("cuda:0")
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    lat = np.array(r["lat"])
    out = {
        "metric": METRIC,
        "value": round(m / (ms_step * 1e-3) / 1e9, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "beta": r["beta"], "graph_seed": 1, "shift_seed": 1,
                   "engine": {0: "auto", 1: "persistent", 2: "launch", 3: "workgroup", 4: "team"}.get(args.engine, "?"),
                   "parallelism": "single-gpu"},
        "decompositions_per_s": round(1e3 / ms_step, 3),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
        "bit_exact": r["bit_exact"],
        "rounds": stats["rounds"], "td_rounds": stats["td_rounds"], "bu_rounds": stats["bu_rounds"],
        "tail_sweeps": stats["tail_iters"],
        "arcs_examined": stats["arcs_examined"],
        "examined_arcs_per_s": round(stats["arcs_examined"] / (ms_step * 1e-3), 1),
        "stage_ms": {k: round(stats[k], 4) for k in ("ms_prep", "ms_rounds", "ms_finalize", "ms_cut")},
        "roofline": roofline_block(stats, n, round_kernel(stats, args.engine),
                                   measured_traffic(args.workload, round_kernel(stats, args.engine))),
    }
    if not args.no_grids:
        out["grid2d"] = run_grid2d(ldd)
        out["grid3d"] = run_grid3d(ldd)
        out["shift_variants"] = run_shift_variants(ldd)
    if not args.no_batch:
        torch.cuda.empty_cache()
        out["batched"] = run_batched(reps=5)
    if not args.no_serve:
        torch.cuda.empty_cache()
        out["served"] = run_serving(args.serve_requests)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.workload} ...")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
