"""Benchmark: exact k-clique counting, k = 3..8, on a seeded Chung-Lu power-law
graph (n = 1,000,000, m = 20,000,000, exponent 2.1, weight cap 10^4), plain
persistent kernel on one MI355X.

One step = the whole counting path over the device-resident CSR: load and
validate it (dm_load_csr, device to device), orient it by (degree, id) rank,
then count k-cliques for every k in 3..8 (dm_count_cliques).  The metric is
enumerated subgraphs per second: the sum of the six exact counts divided by
the step time.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KS = (3, 4, 5, 6, 7, 8)
# Counters of the k=8 clique_kernel launch on the benchmark graph, from
# rocprofv3 --pmc passes over `bench.py --steps 1 --warmup 0 --no-cpu-baseline
# --no-extras` (the profile named below): VALU wave instructions per launch
# (SQ_INSTS_VALU) and HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, each
# scaled by what the counter reads for a device copy of known size).  Valid
# only for the kernel source they were taken on.
CLIQUE_K8 = {"source_sha": "d6e1706eb4102345", "valu_insts": 618152677106.0,
             "active_lane_fraction": 18407614113773.0 / (64 * 618152677106.0),
             "hbm_bytes": 2.0 * 710069.25 * 1024 + 214022.6875 * 1024,
             "profile": "profiles/clique_kernel_cl1m_k8_counters.md"}


def kernel_source_sha(kernel: str = "dm_clique.hip") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in (kernel, "dm_device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2212_04551_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# Counters of the motif kernel's timed launch on the sampled 5-motif workload
# (same passes and scaling), valid only for the kernel source they were taken on.
MOTIF_K5 = {"source_sha": "d29dfb677d40ed31", "valu_insts": 891021959665.0,
            "active_lane_fraction": 28826449997317.0 / (64 * 891021959665.0),
            "hbm_bytes": 2.0 * 241171174.9375 * 1024 + 55297142.46875 * 1024,
            "profile": "profiles/motif_kernel_cl100k_k5_sample_counters.md"}
# MI355X VALU issue peak: 256 CUs x 4 SIMDs, a wave64 VALU instruction takes
# 4 cycles on a 16-lane SIMD, at 2.4 GHz: 6.14e11 wave instructions/s, i.e.
# 39.3e12 lane operations/s.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_info():
    """Host CPU: logical CPUs, the CPUs this process may run on, the model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"nproc": os.cpu_count() or 1, "affinity": aff, "model": model}


# The GPU host's share of CPUs per GPU: the oracle never runs more threads.
HOST_THREADS_CAP = 16


def cpu_baseline(g, budget_s: float, seed: int = 0):
    """The oracle (plain rank-ordered backtracking) on a bounded sample: for each
    k, the roots of one seeded uniform permutation are enumerated in order for
    a fixed wall-clock slice (threads abandon their current root at the
    deadline; everything found until then is counted).  Run on every CPU this
    process may use (at most HOST_THREADS_CAP), then on one thread."""
    import oracle as O

    info = cpu_info()
    threads = max(1, min(info["affinity"], HOST_THREADS_CAP))
    order = np.random.default_rng(seed).permutation(g.n).astype(np.int32)

    def run(nthreads, per_k):
        found, used, roots = 0, 0.0, {}
        for k in KS:
            f, started, el = O.clique_timed(g, k, order, nthreads, per_k)
            found += f
            used += el
            roots[k] = started
            log(f"cpu baseline ({nthreads} threads) k={k}: {f} cliques from {started} roots in {el:.2f}s")
        return (found / used if used > 0 else 0.0), roots

    multi_s = 0.8 * budget_s / len(KS)
    single_s = 0.2 * budget_s / len(KS)
    v_multi, roots_multi = run(threads, multi_s)
    v_single, roots_single = run(1, single_s)
    return {
        "value": v_multi,
        "unit": "subgraphs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"each k=3..8: roots of one seeded uniform permutation enumerated in order for {multi_s:.1f}s "
                  f"wall-clock on {threads} threads (roots begun per k: {roots_multi}); same graph as the GPU run",
        "single_thread_value": v_single,
        "single_thread_sample": f"the same permutation, {single_s:.1f}s per k on 1 thread (roots begun: {roots_single})",
        "nproc": info["nproc"],
        "affinity_cpus": info["affinity"],
        "cpu_model": info["model"],
        "threads_note": f"all CPUs this process may use, capped at {HOST_THREADS_CAP} (the GPU host's CPU share per GPU)",
    }


def base_record(metric_value, ms_per_step, steps, warmup, workload, extra_config, dtype="u64"):
    return {
        "metric": "enumerated subgraphs/s (k-clique, k-motif), learned+batched vs plain, exact",
        "value": metric_value,
        "unit": "subgraphs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": dict({"workload": workload}, **extra_config),
    }


def device_info():
    """The GPU and software the line was measured on."""
    import torch
    p = torch.cuda.get_device_properties(0)
    info = {"name": p.name, "arch": getattr(p, "gcnArchName", ""), "compute_units": p.multi_processor_count,
            "memory_GiB": round(p.total_memory / 2**30, 1), "hip": getattr(torch.version, "hip", None),
            "torch": torch.__version__}
    try:
        from paper_2212_04551_amd import dm
        info["library"] = os.path.relpath(dm.LIB_PATH, ROOT)
    except Exception:  # noqa: BLE001 - informational only
        pass
    return info


def timed_steps(fn, steps, warmup, label):
    import torch
    for w in range(warmup):
        t = time.perf_counter()
        fn()
        log(f"{label} warmup {w}: {time.perf_counter() - t:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        r = fn()
        log(f"{label} step {s} done")
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) * 1e3 / steps


def copy_probe():
    """One 1 GiB device-to-device copy: the calibration kernel of known size
    for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def idle_fraction(ws):
    w = ws.view(-1, 4).cpu().numpy().astype(np.float64)
    w = w[w[:, 0] + w[:, 1] > 0]
    tot = w[:, 0].sum() + w[:, 1].sum()
    return float(w[:, 1].sum() / tot) if tot > 0 else 0.0


def train_model(make_graph, seeds, op, k, epochs, batch=4096, lr=1e-3, sample=1.0):
    """Record per-root tree sizes with the plain kernel on `seeds` (on a seeded
    `sample` fraction of each graph's roots), then train the MLP on the GPU."""
    import torch
    from paper_2212_04551_amd import dm
    feats, targets = [], []
    t0 = time.perf_counter()
    for sd in seeds:
        g = make_graph(sd)
        h = dm.load_graph(g)
        roots = None
        if sample < 1.0:
            roots = np.sort(np.random.default_rng(1000 + sd).choice(g.n, max(1, int(g.n * sample)),
                                                                     replace=False)).astype(np.int32)
        rows = g.n if roots is None else len(roots)
        stats = torch.zeros((rows, 3), dtype=torch.int64, device="cuda")
        if op == "motif":
            dm.count_motifs(h, k, root_stats=stats, roots=roots)
        else:
            dm.count_cliques(h, k, root_stats=stats, roots=roots)
        F = dm.features(h)
        if roots is not None:
            F = F[torch.from_numpy(roots.astype(np.int64)).cuda()].contiguous()
        feats.append(F)
        targets.append(dm.mlp_targets(stats))
        log(f"recorded seed {sd}: n={g.n} roots={rows} ({time.perf_counter() - t0:.1f}s)")
    t_rec = time.perf_counter() - t0
    F = torch.cat(feats)
    T = torch.cat(targets)
    p = dm.mlp_new(0)
    dm.mlp_fit_normalizer(p, F)
    t1 = time.perf_counter()
    hist = dm.mlp_train(p, F, T, epochs=epochs, batch=batch, lr=lr, seed=0)
    t_train = time.perf_counter() - t1
    pred = dm.mlp_forward(p, F).cpu().numpy()
    corr = float(np.corrcoef(pred, T.cpu().numpy())[0, 1])
    log(f"trained: rows={F.shape[0]} loss {hist[0]:.3f} -> {hist[-1]:.3f} corr={corr:.3f}")
    return p, {"rows": int(F.shape[0]), "root_sample": sample, "record_s": t_rec, "train_s": t_train,
               "epochs": epochs, "loss_first": float(hist[0]), "loss_last": float(hist[-1]), "train_corr": corr}


# ---------------------------------------------------------------- workloads

def wl_cl1m_clique(args):
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    t0 = time.perf_counter()
    g, i0 = gg.chung_lu(1_000_000, 20_000_000, 2.1, 1.0e4, args.seed)
    log(f"graph generated in {time.perf_counter() - t0:.1f}s: n={g.n} m={g.m} max_deg={int(g.degrees().max())}")
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(record_events=None):
        h = dm.load_csr(g.n, rp, col, device=True, stream=stream)
        counts = {}
        for k in KS:
            if record_events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            counts[k] = dm.count_cliques(h, k, stream=stream)
            if record_events is not None:
                e1.record(stream)
                record_events.setdefault(k, []).append((e0, e1))
        h.close()
        return counts

    if args.copy_probe:
        copy_probe()

    for w in range(args.warmup):
        t = time.perf_counter()
        counts = step()
        log(f"warmup step {w}: {time.perf_counter() - t:.2f}s counts={counts}")

    events = {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        counts = step(events)
        log(f"step {s} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    total = sum(counts.values())
    value = total / (ms_per_step / 1e3)

    # dominant launch: k = 8.  Its roofline is the VALU issue rate: the
    # launch's VALU instructions (SQ_INSTS_VALU, counted by rocprofv3 on this
    # kernel source and workload) x 64 lanes / the launch's HIP-event time.
    kmax = max(KS)
    per_k_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in events[k]])) for k in KS}
    t8 = per_k_ms[kmax] / 1e3
    out = base_record(value, ms_per_step, args.steps, args.warmup,
                      "k-clique counting k=3..8, Chung-Lu n=1e6 m=2e7 gamma=2.1 wmax=1e4 seed 0, "
                      "degree-ordered DAG, plain persistent kernel",
                      {"n": g.n, "m": g.m, "k": list(KS), "counts": {str(k): int(v) for k, v in counts.items()},
                       "per_k_ms": per_k_ms, "schedule": "plain"})
    fresh = kernel_source_sha() == CLIQUE_K8["source_sha"]
    # Section IV's byte model (each tree node reads its newest vertex's row
    # offsets and out-list once), as a lower bound from the step's own counts:
    # nodes = every j-clique for j = 1..7 (j = 1: n, j = 2: m), and an out-list
    # of a j-clique's newest vertex holds at least its extensions, so the list
    # entries read are at least the (j+1)-clique count.
    nodes = g.n + g.m + sum(counts[j] for j in range(3, kmax))
    entries = g.m + sum(counts[j] for j in range(3, kmax + 1))
    b_model = 8.0 * nodes + 4.0 * entries
    byte_model = {
        "bytes_lower_bound": b_model, "achieved_GBs": b_model / t8 / 1e9,
        "frac_of_hbm_peak": b_model / t8 / 1e9 / HBM_PEAK_GBS,
        "why_not_binding": "each root's bitmap rows are built once (row cache) and every deeper level is an AND + "
                           "popcount over rows held in LDS or L2, so the adjacency reads the model charges per node "
                           "never reach HBM; the counted HBM traffic is the 'traffic' field",
    }
    if fresh:
        lane_ops = 64.0 * CLIQUE_K8["valu_insts"]
        achieved = lane_ops / t8 / 1e12
        out["roofline"] = {
            "bound": "alu", "kernel": "clique_kernel (k=8 launch)",
            "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS,
            "traffic": CLIQUE_K8["hbm_bytes"],
            "basis": f"SQ_INSTS_VALU = {CLIQUE_K8['valu_insts']:.4g} wave instructions per launch x 64 lanes "
                     f"({CLIQUE_K8['profile']}) / this run's HIP-event launch time {per_k_ms[kmax]:.1f} ms; "
                     f"peak = 1024 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU instruction x 64 lanes",
            "active_lane_fraction": CLIQUE_K8["active_lane_fraction"],
            "byte_model": byte_model,
        }
    else:
        # counters stale: the kernel changed since they were taken; fall back
        # to a stated model of 4 VALU ops (64-bit AND + popcount) per j-clique
        # node, j = 2..7, and no traffic figure
        ops = 4.0 * (nodes - g.n)
        achieved = ops / t8 / 1e12
        out["roofline"] = {
            "bound": "alu", "kernel": "clique_kernel (k=8 launch)",
            "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS,
            "traffic": None,
            "basis": "model (counters stale for this kernel source): 4 int32 ops x j-clique nodes, j = 2..7",
            "byte_model": byte_model,
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_budget)
    if not args.no_extras:
        del rp, col
        torch.cuda.empty_cache()
        out["configs"] = extra_configs(args)
    return out


def measure_er516(args):
    """Induced 4-motifs on G(516, 1200) seed 0, plain: per-call time including
    the device-to-device load of the CSR (launch-latency bound)."""
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    g = gg.workload_graph("er516", args.seed)
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()

    def step():
        h = dm.load_csr(g.n, rp, col, device=True)
        c = dm.count_motifs(h, 4)
        h.close()
        return c

    steps = max(args.steps, 20)
    c, ms = timed_steps(step, steps, max(args.warmup, 1), "er516")
    return {"value": int(c.sum()) / (ms / 1e3), "unit": "subgraphs/s", "ms_per_call": ms, "calls": steps,
            "subgraphs": int(c.sum()), "counts": [int(x) for x in c], "schedule": "plain",
            "note": "launch-latency bound: 35k subgraphs per call, load of the CSR included"}


def wl_er516_motif(args):
    r = measure_er516(args)
    return base_record(r["value"], r["ms_per_call"], r["calls"], args.warmup,
                       "induced 4-motif counting, G(n=516, m=1200) seed 0, plain",
                       {"counts": r["counts"], "note": r["note"]})


def wl_cl100k_learned(args):
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    # weight caps: sqrt(2m) for k = 5; for k = 6 a cap that keeps the total near 1e13
    caps = {5: 1414.0, 6: 120.0}
    results = {}
    total_plain = total_learned = 0.0
    subgraphs = 0
    for k, cap in caps.items():
        make = lambda sd, cap=cap: gg.chung_lu(100_000, 1_000_000, 2.3, cap, sd)[0]
        model, tinfo = train_model(make, range(1, 11), "motif", k, epochs=args.epochs, sample=0.1)
        g = make(0)
        rp = torch.from_numpy(g.row_ptr).cuda()
        col = torch.from_numpy(g.col).cuda()
        ws = torch.zeros(256 * 32 * 4, dtype=torch.int64, device="cuda")
        warm_roots = np.arange(0, g.n, 100, dtype=np.int32)

        def run(sched, mlp=None, roots=None):
            def step():
                h = dm.load_csr(g.n, rp, col, device=True)
                c = dm.count_motifs(h, k, sched=sched, mlp=mlp, wave_stats=ws, roots=roots)
                h.close()
                return c
            return step

        # each full run takes about a minute or more: one warm-up on a 1% root
        # sample, then single timed runs (idle fractions from the same runs)
        run(dm.DM_SCHED_PLAIN, roots=warm_roots)()
        ws.zero_()
        cp, ms_plain = timed_steps(run(dm.DM_SCHED_PLAIN), 1, 0, f"motif k={k} plain")
        idle_plain = idle_fraction(ws)
        ws.zero_()
        cl, ms_learned = timed_steps(run(dm.DM_SCHED_LEARNED, model), 1, 0, f"motif k={k} learned")
        idle_learned = idle_fraction(ws)
        assert np.array_equal(cp, cl), "learned ordering changed a count"
        n_sub = int(cp.sum())
        results[str(k)] = {"weight_cap": cap, "max_degree": int(g.degrees().max()), "subgraphs": n_sub,
                           "plain_ms": ms_plain, "learned_ms": ms_learned, "speedup": ms_plain / ms_learned,
                           "idle_plain": idle_plain, "idle_learned": idle_learned, "training": tinfo,
                           "counts": [int(x) for x in cp]}
        log(f"k={k}: {n_sub} subgraphs, plain {ms_plain:.0f} ms, learned {ms_learned:.0f} ms")
        total_plain += ms_plain
        total_learned += ms_learned
        subgraphs += n_sub
    out = base_record(subgraphs / (total_learned / 1e3), total_learned, 1, 0,
                      "induced k-motif counting k=5 (weight cap 1414) and k=6 (weight cap 120), Chung-Lu n=1e5 m=1e6 "
                      "gamma=2.3 seed 0, learned ordering (MLP trained on 10% root samples of seeds 1..10) vs plain; "
                      "single timed runs",
                      {"per_k": results, "plain_value": subgraphs / (total_plain / 1e3),
                       "speedup_learned_vs_plain": total_plain / total_learned})
    return out


def wl_cl100k_motif_sample(args):
    """5-motifs on the cl100k graph (weight cap 1414), a seeded 5% root sample:
    the motif kernel alone, with its HBM roofline."""
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    g = gg.chung_lu(100_000, 1_000_000, 2.3, 1414.0, args.seed)[0]
    roots = np.sort(np.random.default_rng(7).choice(g.n, g.n // 20, replace=False)).astype(np.int32)
    h = dm.load_graph(g)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        copy_probe()
    # algorithmic bytes: every expanded node reads its newest vertex's row_ptr
    # pair (16 B) and adjacency (4 B per entry), from an untimed record run
    stats = torch.zeros((len(roots), 3), dtype=torch.int64, device="cuda")
    ref = dm.count_motifs(h, 5, roots=roots, root_stats=stats)
    st = stats.cpu().numpy().astype(np.float64)
    nodes, reads = st[:, 0].sum(), st[:, 2].sum()
    alg_bytes = 16.0 * nodes + 4.0 * reads
    for _ in range(args.warmup):
        dm.count_motifs(h, 5, roots=roots, stream=stream)
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        c = dm.count_motifs(h, 5, roots=roots, stream=stream)
        e1.record(stream)
        evs.append((e0, e1))
        log(f"step {s_} done")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    assert np.array_equal(c, ref)
    kms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    n_sub = int(c.sum())
    out = base_record(n_sub / (ms / 1e3), ms, args.steps, args.warmup,
                      "induced 5-motif counting, Chung-Lu n=1e5 m=1e6 gamma=2.3 weight cap 1414 seed 0, "
                      "seeded 5% root sample (5000 roots), plain",
                      {"subgraphs": n_sub, "roots": int(len(roots)), "tree_nodes": int(nodes),
                       "adjacency_reads": int(reads), "kernel_ms": kms})
    achieved = alg_bytes / (kms / 1e3) / 1e9
    byte_model = {"bytes": alg_bytes, "achieved_GBs": achieved, "frac_of_hbm_peak": achieved / HBM_PEAK_GBS,
                  "work": f"16 B x {int(nodes)} tree nodes + 4 B x {int(reads)} adjacency entries"}
    if kernel_source_sha("dm_motif.hip") == MOTIF_K5["source_sha"]:
        # the nearer ceiling is VALU issue (about half of it is used); HBM
        # traffic counted per launch is a few percent of its peak
        ops = 64.0 * MOTIF_K5["valu_insts"] / (kms / 1e3) / 1e12
        out["roofline"] = {
            "bound": "alu", "kernel": "motif_kernel", "achieved": ops, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": ops / ALU_PEAK_TOPS, "traffic": MOTIF_K5["hbm_bytes"],
            "basis": f"SQ_INSTS_VALU = {MOTIF_K5['valu_insts']:.4g} per launch x 64 lanes ({MOTIF_K5['profile']}) "
                     f"/ this run's HIP-event launch time {kms:.1f} ms",
            "active_lane_fraction": MOTIF_K5["active_lane_fraction"],
            "hbm_counted_GBs": MOTIF_K5["hbm_bytes"] / (kms / 1e3) / 1e9,
            "byte_model": byte_model,
        }
    else:
        out["roofline"] = {"bound": "hbm", "kernel": "motif_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "basis": "byte model (counters stale for this kernel source)", "byte_model": byte_model}
    return out


def measure_batch4096(args, steps):
    """Batched induced 5-motifs over 4096 graphs: the autotuned captured
    batch launch against one plain call per graph (both warm: every graph's
    rank-renamed copy and the batch's union exist before timing)."""
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    t0 = time.perf_counter()
    graphs = [gg.batch_graph(i) for i in range(4096)]
    calib = [gg.batch_graph(4096 + i) for i in range(256)]
    hs = [dm.load_graph(g) for g in graphs]
    hc = [dm.load_graph(g) for g in calib]
    log(f"4096 + 256 graphs generated and loaded in {time.perf_counter() - t0:.1f}s; "
        f"n total {sum(g.n for g in graphs)}, m total {sum(g.m for g in graphs)}")
    t1 = time.perf_counter()
    tune = dm.autotune(hc, dm.DM_OP_MOTIF, 5)
    t_tune = time.perf_counter() - t1
    log(f"autotuned on 256 calibration graphs (seeds 4096..4351) in {t_tune:.1f}s: {tune}")
    t2 = time.perf_counter()
    first = dm.batch(hs, dm.DM_OP_MOTIF, 5, sched=dm.DM_SCHED_AUTOTUNE)  # builds the union, captures the launch
    t_setup = time.perf_counter() - t2
    cb, ms_batch = timed_steps(lambda: dm.batch(hs, dm.DM_OP_MOTIF, 5, sched=dm.DM_SCHED_AUTOTUNE),
                               steps, 1, "batch autotuned")
    cbu, ms_untuned = timed_steps(lambda: dm.batch(hs, dm.DM_OP_MOTIF, 5), steps, 1, "batch untuned")

    def plain():
        return np.stack([dm.count_motifs(h, 5) for h in hs])

    cpl, ms_plain = timed_steps(plain, 1, 1, "plain per-graph")
    assert np.array_equal(cb, cpl) and np.array_equal(first, cb) and np.array_equal(cbu, cb), \
        "batch counts differ from per-graph counts"
    n_sub = int(cb.sum())
    return {"value": n_sub / (ms_batch / 1e3), "unit": "subgraphs/s", "subgraphs": n_sub,
            "batched_autotuned_ms": ms_batch, "batched_untuned_ms": ms_untuned, "plain_per_graph_ms": ms_plain,
            "plain_value": n_sub / (ms_plain / 1e3), "speedup_vs_plain": ms_plain / ms_batch,
            "tuning": tune, "tune_s": t_tune, "tuned_on": "256 calibration graphs, seeds 4096..4351",
            "first_call_setup_s": t_setup}


def wl_batch4096(args):
    r = measure_batch4096(args, args.steps)
    return base_record(r["value"], r["batched_autotuned_ms"], args.steps, 1,
                       "batched induced 5-motif counting over 4096 graphs (n~U{20..2000}; even: G(n,m) d~U[4,16); "
                       "odd: BA m0~U{2..6}), one hipGraph-captured persistent launch, autotuned vs plain per-graph",
                       {k: v for k, v in r.items() if k not in ("value", "unit")})


def measure_sbm(args, steps):
    """Large-k cliques (k = 10..12) on the 200 x 60 planted-community SBM,
    seed 0: plain against learned ordering + autotuned knobs.  The MLP is
    trained on tree sizes recorded on seeds 1..10 (k = 12); the knobs are
    tuned per k on seed 11 with the learned queue.  Counts are 0 here, so the
    throughput is tree nodes per second: the nodes the counting launch expands
    in its wave DFS (wave_stats; nodes expanded inside the per-lane solver are
    not counted, so this is a lower bound on the nodes it visits)."""
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    make = lambda sd: gg.sbm(200, 60, 0.45, 0.0005, sd)
    model, tinfo = train_model(make, range(1, 11), "clique", 12, epochs=args.epochs, batch=1024)
    hcal = dm.load_graph(make(11))
    g = make(0)
    h = dm.load_graph(g)
    ws = torch.zeros(256 * 32 * 4, dtype=torch.int64, device="cuda")
    per = {}
    tot_plain = tot_learned = 0.0
    nodes_total = 0
    for k in (10, 11, 12):
        tune = dm.autotune([hcal], dm.DM_OP_CLIQUE, k, sched=dm.DM_SCHED_LEARNED, mlp=model)
        ws.zero_()
        cp, msp = timed_steps(lambda: dm.count_cliques(h, k, wave_stats=ws), steps, 1, f"sbm k={k} plain")
        nodes = int(ws.view(-1, 4)[:, 2].sum().item())  # the last launch's (each launch overwrites its rows)
        cl, msl = timed_steps(lambda: dm.count_cliques(h, k, sched=dm.DM_SCHED_LEARNED | dm.DM_SCHED_AUTOTUNE,
                                                       mlp=model), steps, 1, f"sbm k={k} learned")
        assert cp == cl
        per[str(k)] = {"count": int(cp), "dfs_nodes": nodes, "plain_ms": msp, "learned_autotuned_ms": msl,
                       "speedup": msp / msl, "tuning": tune}
        tot_plain += msp
        tot_learned += msl
        nodes_total += nodes
    return {"value": nodes_total / (tot_learned / 1e3), "unit": "tree nodes/s (wave DFS nodes, lower bound)",
            "plain_value": nodes_total / (tot_plain / 1e3), "speedup_vs_plain": tot_plain / tot_learned,
            "per_k": per, "training": tinfo, "tuned_on": "seed 11 (training seeds 1..10, evaluation seed 0)"}


def wl_sbm_largek(args):
    r = measure_sbm(args, args.steps)
    out = base_record(r["value"], sum(v["learned_autotuned_ms"] for v in r["per_k"].values()), args.steps, 1,
                      "k-clique counting k=10..12, SBM 200 blocks x 60, p_in 0.45, p_out 0.0005, seed 0; "
                      "learned + autotuned vs plain; value is tree nodes/s (the counts are 0 or near 0)",
                      {k: v for k, v in r.items() if k not in ("value", "unit")})
    out["unit"] = r["unit"]
    return out


def wl_ablation(args):
    """Section V-A ablation on MI355X: DFS (one lane per traversal,
    DM_IMPL_DFS), WC (wave per traversal, static schedule: DM_NO_DONATION),
    HOST (wave per traversal with the paper's own load balancing: the launch
    stopped, its untried work copied to the host, split and relaunched,
    DM_SCHED_HOST_BALANCE) and OPT (wave per traversal with in-kernel
    donation, the default), timed with
    HIP events on the benchmark graphs: cliques k = 3..6 on the 10^6-vertex
    Chung-Lu graph, motifs k = 3, 4 on the 10^5-vertex Chung-Lu graph (weight
    cap 1414) and k = 5 at weight cap 200.  Counts must agree across the
    three.  A DFS run longer than --ablation-limit seconds stops the DFS
    column for the larger k of that operation (marked null)."""
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    stream = torch.cuda.current_stream()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    impls = (("DFS", dm.DM_IMPL_DFS), ("WC", dm.DM_NO_DONATION), ("HOST", dm.DM_SCHED_HOST_BALANCE),
             ("OPT", dm.DM_SCHED_PLAIN))
    only = set(args.ablation_only.split(",")) if args.ablation_only else None
    rows = []
    series = [("clique", "cl1m", lambda: gg.chung_lu(1_000_000, 20_000_000, 2.1, 1.0e4, args.seed)[0], (3, 4, 5, 6)),
              ("motif", "cl100k_cap1414", lambda: gg.chung_lu(100_000, 1_000_000, 2.3, 1414.0, args.seed)[0], (3, 4)),
              ("motif", "cl100k_cap200", lambda: gg.chung_lu(100_000, 1_000_000, 2.3, 200.0, args.seed)[0], (5,))]
    dfs_ok = {"clique": True, "motif": True}  # per operation, across its graphs (larger k follow)
    for op, gname, make, ks in series:
        if only and not any(x.startswith(f"{op}{k}") for x in only for k in ks):
            continue
        g = make()
        h = dm.load_graph(g, orient=(op == "clique"), rank=(op == "motif"))
        for k in ks:
            row = {"op": op, "graph": gname, "k": k}
            ref = None
            for name, flag in impls:
                if only and f"{op}{k}{name}" not in only:
                    continue
                if name == "DFS" and not dfs_ok[op]:
                    row[name + "_ms"] = None
                    continue
                fn = (lambda f=flag: dm.count_cliques(h, k, sched=f, stream=stream)) if op == "clique" else \
                     (lambda f=flag: dm.count_motifs(h, k, sched=f, stream=stream))
                fn()  # warm-up (row cache, dictionary, workspace)
                c, ms = timed(fn)
                tot = int(c) if op == "clique" else int(np.asarray(c).sum())
                if ref is None:
                    ref = c
                assert np.array_equal(np.asarray(c), np.asarray(ref)), (op, k, name)
                row[name + "_ms"] = ms
                extra = ""
                if name == "HOST":
                    row["HOST_launches"] = dm.last_launch_count()
                    extra = f", {row['HOST_launches']} launches"
                row["subgraphs"] = tot
                log(f"ablation {op} {gname} k={k} {name}: {ms:.1f} ms ({tot} subgraphs{extra})")
                if name == "DFS" and ms > 1e3 * args.ablation_limit:
                    dfs_ok[op] = False
            for a, b in (("DFS", "WC"), ("WC", "OPT"), ("DFS", "OPT"), ("WC", "HOST"), ("HOST", "OPT")):
                if row.get(a + "_ms") and row.get(b + "_ms"):
                    row[f"{a}/{b}"] = row[a + "_ms"] / row[b + "_ms"]
            rows.append(row)
        h.close()
        del g
    best = [r for r in rows if r.get("OPT_ms")]
    tot_sub = sum(r["subgraphs"] for r in best)
    tot_ms = sum(r["OPT_ms"] for r in best)
    out = base_record(tot_sub / (tot_ms / 1e3) if tot_ms else 0.0, tot_ms, 1, 1,
                      "ablation (Section V-A): DFS one lane per traversal vs WC wave per traversal without load "
                      "balancing vs HOST stop/copy/relaunch balancing vs OPT in-kernel donation; cliques k=3..6 on "
                      "Chung-Lu n=1e6 m=2e7, motifs "
                      "k=3,4 on Chung-Lu n=1e5 m=1e6 cap 1414 and k=5 at cap 200",
                      {"rows": rows})
    return out


def wl_directed(args):
    """Directed induced motifs (dm_count_motifs_directed), k = 3..5, on an
    orientation of a 10^5-vertex Chung-Lu graph (m = 5*10^5, exponent 2.3,
    weight cap 100; each edge one arc, a fair coin for its direction, both arcs
    with probability 0.2); warm launches timed with HIP events; the directed
    class counts must sum to the undirected motif count of the same handle."""
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    stream = torch.cuda.current_stream()
    if args.copy_probe:
        copy_probe()
    rows = []
    for gname, ks in (("cl100k_m5e5_cap100", (3, 4, 5)),):
        d = gg.orient(gg.chung_lu(100_000, 500_000, 2.3, 100.0, args.seed)[0], args.seed + 1, both=0.2)
        h = dm.load_digraph(d)
        for k in ks:
            dm.count_motifs_directed(h, k, stream=stream)
            ms = []
            for _ in range(max(1, args.steps)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(stream)
                c = dm.count_motifs_directed(h, k, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            u = dm.count_motifs(h, k, stream=stream)
            assert int(c.sum()) == int(u.sum()), (gname, k)
            t = float(np.median(ms))
            rows.append({"graph": gname, "arcs": d.arcs, "k": k, "ms": t, "subgraphs": int(c.sum()),
                         "classes_seen": int((c > 0).sum()), "subgraphs_per_s": c.sum() / (t / 1e3)})
            log(f"directed {gname} k={k}: {t:.1f} ms, {int(c.sum())} subgraphs, {int((c > 0).sum())} classes seen")
        h.close()
    tot = sum(r["subgraphs"] for r in rows)
    tms = sum(r["ms"] for r in rows)
    return base_record(tot / (tms / 1e3), tms, args.steps, 0,
                       "directed induced motifs k=3..5 on an oriented Chung-Lu graph n=1e5 m=5e5 gamma=2.3 cap 100, "
                       "both arcs with probability 0.2", {"rows": rows})


def greedy_makespan(sizes, waves):
    """Greedy list scheduling of roots in the given order onto `waves`
    waves (each idle wave takes the next root): the finish time of the last
    wave, in the units of `sizes`.  What a launch without donation does."""
    import heapq
    h = [0.0] * waves
    for s in sizes:
        heapq.heappush(h, heapq.heappop(h) + float(s))
    return max(h)


def rank_order(g):
    """Vertices in (degree, id) rank order: the plain queue's order."""
    deg = g.degrees()
    return np.lexsort((np.arange(g.n), deg))


def wl_ordering(args):
    """What the learned root order can gain, per configuration: the plain
    queue (rank order), the MLP's order and the order by the recorded tree
    sizes themselves (a perfect predictor, DM_SCHED_COST), each launched with
    and without in-kernel donation; wave idle fractions from wave_stats; and,
    from the recorded per-root tree nodes, the greedy makespan of each order
    on the launch's waves beside the ideal max(total / waves, largest root)."""
    import torch
    from paper_2212_04551_amd import dm
    from paper_2212_04551_amd import graphgen as gg

    stream = torch.cuda.current_stream()
    ws = torch.zeros(256 * 32 * 4, dtype=torch.int64, device="cuda")

    def launch(h, op, k, **kw):
        fn = dm.count_cliques if op == "clique" else dm.count_motifs
        fn(h, k, stream=stream, **kw)  # warm (queues, caches)
        ws.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        c = fn(h, k, stream=stream, wave_stats=ws, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        w = ws.view(-1, 4).cpu().numpy().astype(np.float64)
        w = w[w[:, 0] + w[:, 1] > 0]
        return c, e0.elapsed_time(e1), float(w[:, 1].sum() / max(1.0, w[:, :2].sum())), int(len(w))

    def study(name, g, h, op, k, model, cost_k):
        stats = torch.zeros((g.n, 3), dtype=torch.int64, device="cuda")
        (dm.count_cliques if op == "clique" else dm.count_motifs)(h, cost_k, root_stats=stats)
        nodes = stats[:, 0].cpu().numpy().astype(np.float64)
        cost = dm.mlp_targets(stats)
        pred = dm.mlp_forward(model, dm.features(h)).cpu().numpy()
        row = {"op": op, "k": k, "cost_from_records_at_k": cost_k}
        ref = None
        for label, kw in (("plain", {}), ("mlp", dict(sched=dm.DM_SCHED_LEARNED, mlp=model)),
                          ("recorded", dict(root_cost=cost))):
            for don, flag in (("donation", 0), ("no_donation", dm.DM_NO_DONATION)):
                kk = dict(kw)
                kk["sched"] = kk.get("sched", 0) | flag
                c, ms, idle, waves = launch(h, op, k, **kk)
                if ref is None:
                    ref = c
                assert np.array_equal(np.asarray(c), np.asarray(ref)), (name, label, don)
                row[f"{label}_{don}_ms"] = ms
                row[f"{label}_{don}_idle"] = idle
                row["waves"] = waves
                log(f"ordering {name} k={k} {label} {don}: {ms:.2f} ms, idle {idle:.3f}")
        W = row["waves"]
        orders = {"plain": rank_order(g), "mlp": np.argsort(-pred, kind="stable"),
                  "recorded": np.argsort(-nodes, kind="stable")}
        mk = {lbl: greedy_makespan(nodes[o], W) for lbl, o in orders.items()}
        ideal = max(nodes.sum() / W, nodes.max())
        row.update({"sim_makespan_nodes": mk, "sim_ideal_nodes": ideal,
                    "sim_headroom_plain": 1.0 - ideal / mk["plain"],
                    "sim_mlp_share_of_headroom": (mk["plain"] - mk["mlp"]) / max(1e-9, mk["plain"] - ideal),
                    "pred_vs_recorded_corr": float(np.corrcoef(pred, cost.cpu().numpy())[0, 1])})
        return row

    out = {}
    # SBM large-k cliques: the MLP trained on seeds 1..10 at k = 12
    make = lambda sd: gg.sbm(200, 60, 0.45, 0.0005, sd)
    model, tinfo = train_model(make, range(1, 11), "clique", 12, epochs=args.epochs, batch=1024)
    g = make(0)
    h = dm.load_graph(g)
    out["sbm200x60_k12"] = study("sbm", g, h, "clique", 12, model, 12)
    out["sbm200x60_k12"]["training"] = tinfo
    # cl1m k = 8 cliques: per-root trees at k = 8 are out of a recording run's
    # reach (10^12 nodes visited one by one), so both the MLP (trained on
    # seeds 1, 2, 10% root samples) and the recorded-size order use k = 5 trees
    make = lambda sd: gg.chung_lu(1_000_000, 20_000_000, 2.1, 1.0e4, sd)[0]
    model, tinfo = train_model(make, (1, 2), "clique", 5, epochs=args.epochs, sample=0.1)
    g = make(0)
    h = dm.load_graph(g)
    out["cl1m_k8"] = study("cl1m", g, h, "clique", 8, model, 5)
    out["cl1m_k8"]["training"] = tinfo
    tot = sum(v["plain_donation_ms"] for v in out.values())
    rec = base_record(0.0, tot, 1, 1, "root-order study: plain vs MLP vs recorded-size order, with and without "
                      "donation (SBM 200x60 k=12; Chung-Lu n=1e6 k=8)", {"studies": out})
    rec["value"] = None
    return rec


def extra_configs(args):
    """The other configurations, measured once each after the headline's timed
    steps (never inside them): G(516, 1200) 4-motifs (plain), the 4096-graph
    batched 5-motifs (batched + autotuned vs plain per-graph) and the SBM
    large-k cliques (learned + autotuned vs plain)."""
    out = {}
    for name, fn in (("er516_motif4_plain", lambda: measure_er516(args)),
                     ("batch4096_motif5_batched_vs_plain", lambda: measure_batch4096(args, 2)),
                     ("sbm200x60_clique_k10_12_learned_vs_plain", lambda: measure_sbm(args, 3))):
        t = time.perf_counter()
        out[name] = fn()
        log(f"{name}: done in {time.perf_counter() - t:.1f}s")
    return out


WORKLOADS = {
    "cl1m-clique": wl_cl1m_clique,
    "er516-motif4": wl_er516_motif,
    "cl100k-motif-learned": wl_cl100k_learned,
    "cl100k-motif5-sample": wl_cl100k_motif_sample,
    "batch4096-motif5": wl_batch4096,
    "sbm-clique-largek": wl_sbm_largek,
    "ablation": wl_ablation,
    "directed-motif": wl_directed,
    "ordering": wl_ordering,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="cl1m-clique", choices=sorted(WORKLOADS))
    ap.add_argument("--epochs", type=int, default=20, help="MLP training epochs (learned workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ablation-limit", type=float, default=60.0,
                    help="ablation: seconds after which DFS runs stop for larger k")
    ap.add_argument("--ablation-only", default="",
                    help="ablation: comma list of op+k+impl to run, e.g. clique6DFS,motif4WC (profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the other configurations measured after the headline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one device copy of 1 GiB (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): sharding the roots over several "
              f"GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    out = WORKLOADS[args.workload](args)
    out["device"] = device_info()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
