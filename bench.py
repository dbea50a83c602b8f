"""Benchmark: betweenness TEPS on MI355X, with the oracle timed beside it.

Default workload (the headline): RMAT scale 16, all sources, the batched
mixed-precision form (hybrid: each level by sparse pulls or by MFMA products,
as the tuner chose before timing; batches of 256 sources) against the plain
FP64 per-source form on the same GPU.

One step = one complete betweenness computation over the workload (forward
sweep, backward sweep and accumulation for every source), inputs resident in
HBM.  TEPS = sources * m / t, m = undirected edges after preprocessing (for
the many-graph workload, the sum over graphs of n_g * m_g).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--form F] [--batch B] [--no-cpu-baseline] [--no-compare]

Other workloads (same JSON schema; used for profiles and design figures):
  er1024   ER n=1024, degree 8, plus a spanning tree, all sources: the plain
           FP64 form, against the sparse form
  er16384  ER n=16384, degree 256, all sources: algebraic form, batch 512,
           against the sparse and hybrid forms
  ws4096   4096 Watts-Strogatz graphs, all sources: one persistent launch
  rmat20w  RMAT-20 with weights U{1..255}, 4096 sampled sources: bucketed
           shortest paths per source
  er16384w4
           the er16384 graph with weights U{1..4}, all sources: the algebraic
           form with one product class per weight (Sec. 3.2), batch 512,
           against the plain form's bucketed per-source sweep
  allpairs16384
           ER n=16384, degree 256: BC over every pair by Algorithm 2 (the
           algebraic form's forward fills all-pairs distances and counts, one
           kernel sums the masked triple terms), against Brandes in the same
           context
  sampled16
           RMAT-16, 1024 sources: distances by Algorithm 1 (Sec. 4.1.1) with a
           uniform sample of ceil(sqrt(n) ln n) vertices and search limit
           ceil(sqrt(n)), output left in HBM, against the exact forward and
           backward of the hybrid form for the same sources

Prints one JSON line.  Profiling runs use --sources N (a bounded prefix of the
sources) and --calibrate-copy (a 1 GiB device-to-device copy at the end, the
reference against which rocprofv3 FETCH_SIZE / WRITE_SIZE are scaled).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "BC TEPS (sources·m/s) on RMAT-16; batched-MFMA vs plain BFS form, same GPU"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFS = 2500.0
MFMA_I8_PEAK_TOPS = 5000.0
# 32-bit integer vector operations: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz
VALU_INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# HIP event pairs on every launch of one source batch in TIMING_SAMPLE during
# the timed steps (batches are alike, so the per-launch averages keep every
# level's share; every launch is counted)
TIMING_SAMPLE = 5

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sparse_rmat16_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_0809_1906_amd", "csrc", "sparse.hip")

WORKLOADS = {
    "er1024": {"form": "plain", "batch": 0, "compare": [("sparse", 256)],
               "desc": "er1024: Erdos-Renyi n=1024, average degree 8, plus a seeded random spanning tree; exact "
                       "all-source BC"},
    "rmat16": {"form": "hybrid", "batch": 256, "compare": [("plain", 0)],
               "desc": "rmat16: RMAT scale 16, edgefactor 16, (a,b,c,d)=(.57,.19,.19,.05), symmetrised, "
                       "deduplicated, largest component; exact all-source BC"},
    "er16384": {"form": "algebraic", "batch": 512, "compare": [("sparse", 512), ("hybrid", 512)],
                "desc": "er16384: Erdos-Renyi n=16384, average degree 256, largest component; exact "
                        "all-source BC"},
    "ws4096": {"form": "many", "batch": 0, "compare": [],
               "desc": "ws4096: 4096 Watts-Strogatz graphs, n ~ U{64..4096}, k=6, p=0.1, seeded per graph; "
                       "exact all-source BC of every graph in one persistent launch"},
    "rmat20w": {"form": "plain", "batch": 0, "compare": [],
                "desc": "rmat20w: RMAT scale 20, edgefactor 16, largest component, weights U{1..255}; BC "
                        "over 4096 sources sampled without replacement"},
    "er16384w4": {"form": "algebraic", "batch": 512, "compare": [("plain", 0)],
                  "desc": "er16384w4: Erdos-Renyi n=16384, average degree 256, largest component, weights "
                          "U{1..4}; exact all-source BC"},
    "sampled16": {"form": "hybrid", "batch": 256, "compare": [],
                  "desc": "sampled16: RMAT scale 16 (as rmat16), 1024 sources and a uniform sample of "
                          "ceil(sqrt(n) ln n) = 2325 vertices, search limit ceil(sqrt(n)) = 217; distances by "
                          "Algorithm 1"},
    "allpairs16384": {"form": "algebraic", "batch": 512, "compare": [],
                      "desc": "allpairs16384: Erdos-Renyi n=16384, average degree 256, largest component; BC "
                              "over every ordered pair by Algorithm 2 from all-pairs distances and counts"},
}

DTYPES = {
    "plain": "u64 counts, f64 dependency state and sums",
    "sparse": "u64 counts, f32 dependency state, f64 sums",
    "hybrid": "u64 counts, f32 dependency state, f64 sums; where chosen, int8 MFMA forward products (7-bit "
              "limbs, i32 sums) and bf16 backward products (f32 sums)",
    "algebraic": "int8 MFMA forward products of 7-bit count limbs with i32 accumulate, bf16 MFMA backward "
                 "products with f32 accumulate, u64 counts, f32 dependency state, f64 sums",
    "many": "u64 counts, f32 dependency state, f64 sums",
    "sampled": "int32 distances (u16 limited-search distances, u64 frontier bitmaps)",
    "allpairs": "u64 counts and int32 distances (forward by int8 MFMA products of 7-bit limbs), u32 mask "
                "arithmetic, f64 terms and sums",
}


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the summary is missing, covers another workload, or
    the kernel source changed since the counters were taken."""
    if workload != "rmat16" or not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256_16") != kernel_source_hash():
        return None
    v = fields.get(f"{kernel}.bytes_per_launch")
    return float(v) if v else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pass_bytes(n: int, m: int) -> int:
    """Bytes one source's sweep must move at minimum per pass in the
    per-source model: the int32 column array once (8m for 2m arcs) and about
    24 B of per-vertex state (row offsets, level, count, dependency and a share
    of the BC update): 8m + 24n per pass, 16m + 48n per source."""
    return 8 * m + 24 * n


def weighted_bytes(n: int, m: int) -> int:
    """Per source, weighted: the forward reads every arc's column (4 B) and
    weight (1 B, the values fit a byte), the backward only the DAG arcs (a few
    percent), plus about 50 B of per-vertex state: 10m + 50n."""
    return 10 * m + 50 * n


def load_workload(name, sources):
    import graphgen as gg
    t0 = time.perf_counter()
    if name == "ws4096":
        gs = gg.ws_batch(4096)
        n = sum(g.n for g in gs)
        m = sum(g.m for g in gs)
        log(f"graphs ws4096: {len(gs)} graphs, sum n={n}, sum m={m}, gen {time.perf_counter() - t0:.1f}s")
        return {"graph": gs, "n": n, "m": m, "src": None, "S": n,
                "work": float(sum(g.n * g.m for g in gs))}
    if name == "rmat20w":
        g, src = gg.rmat20w()
    elif name == "allpairs16384":
        g, src = gg.er16384(), None
    elif name == "sampled16":
        g, src, smp = gg.rmat16_sampled()
        log(f"graph {name} n={g.n} m={g.m} sources={src.size} sample={smp.size} gen {time.perf_counter() - t0:.1f}s")
        return {"graph": g, "n": g.n, "m": g.m, "src": src, "sample": smp, "S": int(src.size),
                "work": float(src.size) * g.m}
    else:
        g = getattr(gg, name)()
        src = None
    log(f"graph {name} n={g.n} m={g.m} max_deg={int(g.degrees().max())} gen {time.perf_counter() - t0:.1f}s")
    if sources > 0:
        src = (np.arange(min(sources, g.n), dtype=np.int32) if src is None else src[:sources])
    S = g.n if src is None else int(src.size)
    return {"graph": g, "n": g.n, "m": g.m, "src": src, "S": S, "work": float(S) * g.m}


def host_cpus():
    """(threads the oracle uses, nproc, CPU model).  The oracle uses the CPUs
    this process may run on, at most 16: one GPU's share of a GPU host."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, min(16, avail)), os.cpu_count() or 1, model


def err_report(got, want):
    """max_v |x - y| / max(|y|, 1), its argmax, and the largest purely
    relative error over vertices with BC >= 1."""
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    if want.size == 0:
        return {"max_rel_err_vs_oracle": 0.0}
    e = np.abs(got - want) / np.maximum(np.abs(want), 1.0)
    i = int(np.argmax(e))
    big = np.abs(want) >= 1.0
    pure = float(np.max(np.abs(got - want)[big] / np.abs(want)[big])) if np.any(big) else 0.0
    return {"max_rel_err_vs_oracle": float(e[i]), "argmax_vertex": i, "bc_at_argmax": float(want[i]),
            "max_pure_rel_err_bc_ge_1": pure}


def cpu_baseline(name, wl, target_s: float = 20.0, whole: bool = True):
    """The oracle as it stands, timed on the host: over every source of the
    workload when that fits the budget (else an evenly spaced sample sized to
    about target_s), on the host threads host_cpus() allows; also one thread
    on the first 64 sources.  Returns (baseline dict, oracle BC of the sources
    it ran or None, the sources it ran)."""
    import oracle
    threads, nproc, model = host_cpus()
    cores = {"cores": threads, "nproc": nproc, "cpu_model": model,
             "threads_note": "threads = the CPUs this process may use, at most 16 (one GPU's share of the host)"}
    if name == "ws4096":
        gs = wl["graph"]
        order = list(range(0, len(gs), 3))  # every third graph, in generation order, until the time is up
        t0 = time.perf_counter()
        done, work, per_graph = 0, 0.0, {}
        for i in order:
            per_graph[i] = oracle.bc(gs[i], threads=threads)
            done += 1
            work += gs[i].n * gs[i].m
            if time.perf_counter() - t0 > target_s:
                break
        t = time.perf_counter() - t0
        return ({"value": work / t, "unit": "TEPS", "kind": "oracle", **cores,
                 "sample": f"{done} of {len(gs)} graphs (every third, first ones), all sources each, {threads} "
                           f"threads over sources, {t:.1f} s"}, per_graph, None)
    g = wl["graph"]
    pool = wl["src"] if wl["src"] is not None else np.arange(g.n, dtype=np.int32)
    # one thread, the first 64 sources
    first = pool[:64]
    t0 = time.perf_counter()
    oracle.bc(g, first, threads=1)
    t1 = time.perf_counter() - t0
    single = {"value": first.size * g.m / t1, "unit": "TEPS", "sources": int(first.size), "seconds": t1,
              "sample": f"the first {first.size} sources, one thread"}
    log(f"oracle, one thread, {first.size} sources: {t1:.2f} s")
    est = t1 / max(first.size, 1) * pool.size / threads
    if whole and est <= 3.0 * target_s:
        sample = pool
    else:
        count = int(min(pool.size, max(64, target_s / max(t1 / max(first.size, 1) / threads, 1e-9))))
        sample = pool[np.linspace(0, pool.size - 1, count).astype(np.int64)]
    log(f"oracle on {sample.size} of {pool.size} sources, {threads} threads (estimate {est:.1f} s for all)")
    t0 = time.perf_counter()
    want = oracle.bc(g, sample, threads=threads)
    t = time.perf_counter() - t0
    what = ("every source" if sample.size == pool.size else
            f"{sample.size} of {pool.size} sources (evenly spaced)")
    return ({"value": sample.size * g.m / t, "unit": "TEPS", "kind": "oracle", **cores,
             "sample": f"{what}, serial Brandes per source, {threads} threads over sources, {t:.1f} s",
             "single_core": single}, want, sample)


KERNELS = ("fwd_pull", "bwd_pull", "fwd_push0", "batch_init", "batch_check", "limb_split", "mfma_fwd",
           "coef_split", "mfma_bwd", "plain_sweep", "weighted_sweep", "multigraph_sweep")


def roofline(name, wl, kern, info, steps):
    """Roofline of the dominant kernel: algorithmic bytes (or flops) per
    launch over its average launch time from HIP events in the timed region."""
    dom = max(kern, key=lambda k: kern[k][0])
    ms, launches = kern[dom]
    n, m, S = wl["n"], wl["m"], wl["S"]
    base = {"kernel": dom, "avg_launch_ms": ms / max(launches, 1), "launches": launches,
            "timed": "every launch" if dom in ("plain_sweep", "weighted_sweep", "multigraph_sweep")
            else f"every launch of one source batch in {TIMING_SAMPLE}"}
    if dom in ("mfma_fwd", "mfma_bwd"):
        npad = (n + 255) // 256 * 256
        # with weights 1..M a product runs over K = M * npad (one class each)
        wts = getattr(wl["graph"], "weight", None)
        classes = int(wts.max()) if wts is not None and wts.size else 1
        # the library counts k-tiles of 2^20 flops (one plane's 32 k by 128
        # rows by 128 sources): those multiplied, and those the issued
        # products cover (the rest skipped, every plane's k-tile zero); both
        # count every batch of the timed steps, replayed or host-driven
        if dom == "mfma_fwd":
            run, dense = info.mfma_ktiles_run_fwd, info.mfma_ktiles_dense_fwd
        else:
            run = info.mfma_ktiles_run - info.mfma_ktiles_run_fwd
            dense = info.mfma_ktiles_dense - info.mfma_ktiles_dense_fwd
        executed, issued = float(run) * 2.0 ** 20, float(dense) * 2.0 ** 20
        ach = executed / (ms * 1e-3) / 1e12
        base["weight_classes"] = classes
        base["k_tiles_skipped_frac"] = 1.0 - run / dense if dense else 0.0
        base["issued_dense_tflops"] = issued / (ms * 1e-3) / 1e12
        # the forward's products are int8 (dense peak 5.0 POP/s), the
        # backward's BF16 (2.5 PFLOP/s)
        peak, unit = (MFMA_I8_PEAK_TOPS, "TOP/s") if dom == "mfma_fwd" else (MFMA_BF16_PEAK_TFS, "TFLOP/s")
        return dict(base, bound="mfma", achieved=ach, peak=peak, unit=unit,
                    frac=ach / peak, traffic=None,
                    alg_flops_per_launch=executed / max(launches, 1),
                    planes_equivalent=issued / (2.0 * info.batch * npad * npad * classes),
                    note="executed products: 2^20 flops per k-tile multiplied (one plane's 32 k x 128 rows x "
                         "128 sources); issued_dense_tflops counts the skipped all-zero k-tiles too")
    if dom == "weighted_sweep":
        total = float(S) * steps * weighted_bytes(n, m)
    elif dom == "multigraph_sweep":
        total = float(steps) * sum(g.n * (2 * pass_bytes(g.n, g.m)) for g in wl["graph"])
        base["note"] = "per-source state is LDS-resident; HBM model only"
    elif dom == "plain_sweep":
        total = float(S) * steps * 2 * pass_bytes(n, m)
    else:
        total = float(S) * steps * pass_bytes(n, m)
    ach = total / (ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, name)
    extra = {}
    if traffic:
        # measured DRAM bytes per launch over the launch time, against the
        # peak; and how many algorithmic bytes each DRAM byte served
        extra["dram_frac"] = traffic / (ms / max(launches, 1) * 1e-3) / 1e9 / HBM_PEAK_GBS
        extra["alg_bytes_per_dram_byte"] = total / max(launches, 1) / traffic
        extra["note"] = ("frac = the per-source model's algorithmic bytes (a batch shares its CSR and bitmap "
                         "reads, so one DRAM byte serves several model bytes) per launch time; dram_frac = "
                         "bytes measured by rocprofv3 FETCH_SIZE/WRITE_SIZE per launch time, the HBM rate")
    return dict(base, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                traffic=traffic, alg_bytes_per_launch=total / max(launches, 1), **extra)


def run_allpairs(args, spec, wl, bcgpu, torch):
    """One step = one bc_all_pairs call: the forward fills all-pairs D and
    Lambda, then one kernel sums lambda_sv * lambda_vt / lambda_st over the
    triples with d(s,t) = d(s,v) + d(v,t) (Algorithm 2, Sec. 4.2.1)."""
    g, n, m = wl["graph"], wl["n"], wl["m"]
    form = args.form or spec["form"]
    batch = spec["batch"] if args.batch is None else args.batch
    ctx = bcgpu.BC(g, form=form, batch=batch, timing=True)
    info = ctx.info()
    for i in range(args.warmup):
        ctx.all_pairs()
        log(f"all pairs warmup {i} done")
    ctx.reset()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        got = ctx.all_pairs()
        log(f"all pairs step {i} done")
    dt = (time.perf_counter() - t) / args.steps
    kern = {k: ctx.timing(k) for k in KERNELS + ("all_pairs",) if ctx.timing(k)[1]}
    log("kernel times (ms, launches):", kern)
    ms, launches = kern["all_pairs"]
    avg = ms / launches
    # a tested triple is one three-operand add and half a three-operand
    # minimum: 1.5 VALU lane-instructions, the unit of the peak
    ops = 1.5 * float(n) ** 3
    ach = ops / (avg * 1e-3) / 1e12
    roof = {"kernel": "all_pairs", "avg_launch_ms": avg, "launches": launches, "bound": "alu", "achieved": ach,
            "peak": VALU_INT32_PEAK_TOPS, "unit": "T lane-instructions/s", "frac": ach / VALU_INT32_PEAK_TOPS,
            "traffic": None, "alg_ops_per_launch": ops,
            "note": "n^3 tested triples x 1.5 VALU lane-instructions (v_add3, half a v_min3) per launch; peak = "
                    "256 CUs x 64 lanes x 2.4 GHz lane-instructions/s"}
    compare = {}
    if not args.no_compare:
        ctx.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.run()
        brandes = ctx.read()
        bdt = time.perf_counter() - t
        err = float(np.max(np.abs(got - brandes) / np.maximum(np.abs(brandes), 1.0)))
        compare["brandes_same_context"] = {"value": n * m / bdt, "ms_per_step": bdt * 1e3,
                                           "max_rel_diff_vs_all_pairs": err}
        log(f"brandes {bdt * 1e3:.1f} ms, max rel diff {err:.2e}")
    ctx.close()
    cpu, acc = None, {}
    if not args.no_cpu_baseline:
        cpu, want, _ = cpu_baseline("er16384", wl)
        if want is not None and want.size == n:
            acc = err_report(got, want)
            log(f"all pairs vs oracle: {acc}")
    return {
        "metric": "all-pairs BC by Algorithm 2 on ER-16384, TEPS (n·m/s)",
        "value": n * m / dt,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES["allpairs"],
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n": n, "m": m, "form_filling_D_Lambda": form, "batch": info.batch},
        "compare": compare,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kern.items()},
        "accuracy": acc,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def cpu_baseline_sampled(wl, k: int):
    """The oracle's Algorithm 1 steps on a bounded sample, scaled to the whole
    job: limited searches from 160 evenly spaced distinguished vertices
    (scaled by |S| / 160), Floyd-Warshall on a 1024-vertex H (data-independent
    cost, scaled by (|S| / 1024)^3), and the final minimum for 32 sources over
    those 160 rows (scaled by |S| / 160 and sources / 32).  numpy, one
    thread."""
    from oracle import sampled
    g, src, smp = wl["graph"], wl["src"], wl["sample"]
    S = np.array(list(dict.fromkeys([int(x) for x in src] + [int(x) for x in smp])), np.int64)
    ns, nb, nf, nm = S.size, 160, 1024, 32
    pick = S[np.linspace(0, ns - 1, nb).astype(np.int64)]
    t0 = time.perf_counter()
    Dp = np.stack([sampled.limited_bfs(g, int(x), k) for x in pick])
    t_bfs = (time.perf_counter() - t0) * ns / nb
    H = np.random.default_rng(1).integers(1, 50, size=(nf, nf)).astype(np.int64)
    np.fill_diagonal(H, 0)
    t0 = time.perf_counter()
    DH = sampled.floyd_warshall(H)
    t_fw = (time.perf_counter() - t0) * (ns / nf) ** 3
    t0 = time.perf_counter()
    for r in range(nm):
        np.min(DH[r, :nb][:, None] + Dp, axis=0)
    t_min = (time.perf_counter() - t0) * (ns / nb) * (src.size / nm)
    t = t_bfs + t_fw + t_min
    return {"value": src.size * g.m / t, "unit": "TEPS", "cores": 1, "kind": "oracle",
            "sample": f"limited searches from {nb} of {ns} distinguished vertices ({t_bfs:.1f} s scaled), "
                      f"Floyd-Warshall on a {nf}-vertex H ({t_fw:.1f} s scaled by (|S|/{nf})^3), final minimum "
                      f"for {nm} of {src.size} sources over {nb} rows ({t_min:.1f} s scaled); numpy, one thread; "
                      f"estimated whole job {t:.1f} s"}


def run_sampled(args, spec, wl, bcgpu, torch):
    """One step = one bc_sampled_distances call with the output in HBM:
    limited searches from S, H, Floyd-Warshall, the final minimum
    (Algorithm 1, Sec. 4.1.1)."""
    g, n, m, src, smp = wl["graph"], wl["n"], wl["m"], wl["src"], wl["sample"]
    k = int(np.ceil(np.sqrt(n)))
    ns = len(set(src.tolist()) | set(smp.tolist()))
    sp = (ns + 63) // 64 * 64
    ctx = bcgpu.BC(g, form=args.form or spec["form"], batch=spec["batch"], timing=True)
    out = torch.empty((src.size, n), dtype=torch.int32, device="cuda:0")
    for i in range(args.warmup):
        ctx.sampled_distances(src, smp, k, out=out)
        log(f"sampled warmup {i} done")
    # spot check against exact distances (well inside the w.h.p. regime: k is past the diameter)
    pick = src[:: max(1, src.size // 6)][:6]
    dist, _, _ = ctx.sssp(pick)
    got = out.cpu().numpy()
    rows = [int(np.where(src == p)[0][0]) for p in pick]
    exact_ok = bool(np.array_equal(got[rows], dist))
    log(f"sampled vs exact distances on {len(pick)} sources: {'equal' if exact_ok else 'DIFFERENT'}")
    names = ("limited_bfs", "floyd_warshall", "sampled_min")
    before = {k_: ctx.timing(k_) for k_ in names}
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        ctx.sampled_distances(src, smp, k, out=out)
        log(f"sampled step {i} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / args.steps
    phase = {k_: (ctx.timing(k_)[0] - before[k_][0]) / args.steps for k_ in names}
    log("phase ms per step:", phase)
    # the final minimum is a min-plus product over (source, x, v) terms; in the
    # 16-bit form (taken here: every finite D_H entry is at most the diameter,
    # far below 65534 - k) one packed add and one packed minimum cover two
    # terms per lane, so one VALU lane-instruction per term bounds it
    terms = float(src.size) * ns * n
    ach = terms / (phase["sampled_min"] * 1e-3) / 1e12
    roof = {"kernel": "k_minplus16 (final minimum)", "avg_launch_ms": phase["sampled_min"], "launches": args.steps,
            "bound": "alu", "achieved": ach, "peak": VALU_INT32_PEAK_TOPS, "unit": "Top/s",
            "frac": ach / VALU_INT32_PEAK_TOPS, "traffic": None, "alg_ops_per_launch": terms,
            "note": "sources x |S| x n min-plus terms per launch, one VALU lane-instruction per "
                    "term (v_pk_add_u16 with clamp and v_pk_min_u16, two terms each); peak = 256 CUs x 64 "
                    "lanes x 2.4 GHz"}
    compare = {}
    if not args.no_compare:
        ctx.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run(src)
        ctx.read()
        bdt = time.perf_counter() - t0
        compare["exact_brandes_same_sources"] = {"form": ctx.info().form, "value": src.size * m / bdt,
                                                 "ms_per_step": bdt * 1e3}
        log(f"exact forward+backward for the same sources {bdt * 1e3:.1f} ms")
    ctx.close()
    cpu = None if args.no_cpu_baseline else cpu_baseline_sampled(wl, k)
    return {
        "metric": "sampled-forward distances by Algorithm 1 on RMAT-16, sources·m/s",
        "value": src.size * m / dt,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES["sampled"],
        "data": "synthetic",
        "config": {"workload": spec["desc"], "n": n, "m": m, "sources": int(src.size), "distinguished": ns,
                   "padded": sp, "limit": k, "exact_on_spot_check": exact_ok},
        "compare": compare,
        "phase_ms_per_step": phase,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat16", choices=sorted(WORKLOADS))
    ap.add_argument("--form", default=None, help="form of the measured line (default: the workload's)")
    ap.add_argument("--batch", type=int, default=None, help="batch width (default: the workload's; 0 = tuned)")
    ap.add_argument("--no-compare", "--no-plain", dest="no_compare", action="store_true",
                    help="skip the comparison forms")
    ap.add_argument("--compare-steps", "--plain-steps", dest="compare_steps", type=int, default=1)
    ap.add_argument("--no-free-batch", action="store_true", help="skip the extra run at the tuned batch width")
    ap.add_argument("--edges", action="store_true", help="also accumulate edge betweenness in the measured form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sources", type=int, default=0, help="run only the first N sources (profiling)")
    ap.add_argument("--calibrate-copy", action="store_true", help="end with a 1 GiB device copy")
    ap.add_argument("--host-driven", action="store_true",
                    help="drive every batch of the measured form from the host (no replays; for counter runs)")
    ap.add_argument("--timing", type=int, default=TIMING_SAMPLE,
                    help="HIP events on the launches of one batch in K during the timed steps (0: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (sources shard across GPUs by design, "
                                   "but no multi-GPU path is implemented)"}))
        sys.exit(2)

    import torch

    import paper_0809_1906_amd as bcgpu

    bcgpu.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    spec = WORKLOADS[args.workload]
    form = args.form or spec["form"]
    batch = spec["batch"] if args.batch is None else args.batch
    wl = load_workload(args.workload, args.sources)
    if args.workload == "allpairs16384":
        print(json.dumps(run_allpairs(args, spec, wl, bcgpu, torch)), flush=True)
        return
    if args.workload == "sampled16":
        print(json.dumps(run_sampled(args, spec, wl, bcgpu, torch)), flush=True)
        return
    src, work = wl["src"], wl["work"]

    step_ms = {}

    def timed_runs(form, steps, warmup, batch=0, timing=TIMING_SAMPLE, edges=False, host_driven=False,
                   label=None):
        label = label or form
        t = time.perf_counter()
        ctx = bcgpu.BC(wl["graph"], form="auto" if form == "many" else form, batch=batch, timing=timing,
                       edges=edges, host_driven=host_driven)
        info = ctx.info()
        log(f"{form} create (upload, adjacency bits, tuning) {time.perf_counter() - t:.2f}s: batch {info.batch}, "
            f"products when density >= ({info.mfma_density_fwd:.3f} fwd, {info.mfma_density_bwd:.3f} bwd), "
            f"tuning source {info.tune_source}")
        for i in range(warmup):
            ctx.run(src)
            ctx.read()
            log(f"{label} warmup {i} done")
        ctx.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        per_step = []
        for i in range(steps):
            ts = time.perf_counter()
            ctx.run(src)
            torch.cuda.synchronize()
            per_step.append(time.perf_counter() - ts)
            log(f"{label} step {i} done")
        dt = (time.perf_counter() - t) / steps
        step_ms[label] = {"mean": dt * 1e3, "median": float(np.median(per_step)) * 1e3,
                          "min": float(np.min(per_step)) * 1e3}
        bc = ctx.read()
        log(f"{label} {steps} steps: {dt * 1e3:.1f} ms/step, {work / dt:.3e} TEPS")
        return ctx, dt, bc

    ctx, dt, bc_main = timed_runs(form, args.steps, args.warmup, batch, edges=args.edges, timing=args.timing,
                                  host_driven=args.host_driven)
    main_step_ms = dict(step_ms[form])
    info = ctx.info()
    kern = {}
    for k in KERNELS:
        ms, launches = ctx.timing(k)
        if launches:
            kern[k] = (ms, launches)
    log("kernel times (ms, launches):", kern)
    roof = roofline(args.workload, wl, kern, info, args.steps) if kern else None
    ctx.close()

    free = None
    if form in ("hybrid", "sparse") and batch != 0 and not args.no_free_batch:
        fctx, fdt, _ = timed_runs(form, 1, 1, 0, timing=False)
        finfo = fctx.info()
        fctx.close()
        free = {"batch": finfo.batch, "value": work / fdt, "ms_per_step": fdt * 1e3,
                "mfma_density": [finfo.mfma_density_fwd, finfo.mfma_density_bwd]}

    compare = {}
    if not args.no_compare and form in ("hybrid", "sparse", "algebraic") and args.workload != "er16384w4":
        # the same form with every batch driven level by level from the host
        hctx, hdt, bc_h = timed_runs(form, args.compare_steps, 1, batch, timing=args.timing, host_driven=True,
                                     label="host-driven")
        hctx.close()
        err = float(np.max(np.abs(bc_main / args.steps - bc_h / args.compare_steps) /
                           np.maximum(np.abs(bc_h / args.compare_steps), 1.0)))
        compare["host_driven"] = {"value": work / hdt, "ms_per_step": hdt * 1e3,
                                  "max_rel_diff_vs_measured": err,
                                  "note": "every batch's levels launched from the host, one synchronisation per "
                                          "batch, instead of replaying the recorded batch"}
    if not args.no_compare:
        for cform, cbatch in spec["compare"]:
            # a batched form records its replayed batch in its first step:
            # one untimed step first (the plain form has nothing to record)
            cctx, cdt, bc_c = timed_runs(cform, args.compare_steps, 0 if cform == "plain" else 1, cbatch)
            cinfo = cctx.info()
            ckern = {k: cctx.timing(k)[0] for k in KERNELS if cctx.timing(k)[1]}
            cctx.close()
            # each context accumulated its own number of steps
            per_main, per_c = bc_main / args.steps, bc_c / args.compare_steps
            err = float(np.max(np.abs(per_main - per_c) / np.maximum(np.abs(per_c), 1.0)))
            compare[cform] = {"value": work / cdt, "ms_per_step": cdt * 1e3, "batch": cinfo.batch,
                              "kernel_ms": ckern, "max_rel_diff_vs_measured": err}
            if cform == "plain" and getattr(wl["graph"], "weight", None) is None:
                # the per-source byte model of both passes over the step time
                model = float(wl["S"]) * 2 * pass_bytes(wl["n"], wl["m"])
                compare[cform]["roofline_model_frac"] = model / cdt / 1e9 / HBM_PEAK_GBS
                compare[cform]["roofline_note"] = (
                    "HBM-bound by random sector traffic: rocprofv3 counters on 4096 RMAT-16 sources read "
                    "9.2e11 B (13x the model) at 3.6 TB/s, 0.45 of peak, 19% L2 hits")

    cpu, accuracy = None, {}
    if not args.no_cpu_baseline:
        cpu, want, osrc = cpu_baseline(args.workload, wl)
        per_step = bc_main / args.steps  # the context accumulated every timed step
        if args.workload == "ws4096":
            offs = np.concatenate([[0], np.cumsum([x.n for x in wl["graph"]])])
            worst = {"max_rel_err_vs_oracle": 0.0}
            for i, wv in want.items():
                r = err_report(per_step[offs[i]:offs[i + 1]], wv)
                if r["max_rel_err_vs_oracle"] >= worst["max_rel_err_vs_oracle"]:
                    worst = dict(r, graph=i)
            accuracy = dict(worst, compared=f"{len(want)} graphs, the oracle's CPU-baseline sample")
        elif osrc is not None and (wl["src"] is None and osrc.size == wl["n"]
                                   or wl["src"] is not None and osrc.size == wl["src"].size):
            accuracy = dict(err_report(per_step, want), compared="the measured output, every source")
        elif osrc is not None:
            # the oracle ran a sample: run the same sources on the GPU
            with bcgpu.BC(wl["graph"], form="auto" if form == "many" else form, batch=batch) as sctx:
                sctx.run(osrc)
                accuracy = dict(err_report(sctx.read(), want),
                                compared=f"{osrc.size} sources (the oracle's sample), same form and batch")
        log(f"accuracy vs oracle: {accuracy}")

    if args.calibrate_copy:
        x = torch.empty(256 << 20, dtype=torch.float32, device=dev)  # 1 GiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read, 1 GiB written")

    config = {"workload": spec["desc"], "n": wl["n"], "m": wl["m"], "sources": wl["S"], "batch": info.batch,
              "form": form, "levels_max": info.max_levels, "edge_betweenness": bool(args.edges)}
    if form in ("hybrid", "sparse", "algebraic"):
        config["mfma_density_thresholds"] = [info.mfma_density_fwd, info.mfma_density_bwd]
        config["tune_source"] = ["default", "measured", "cached"][info.tune_source]
        config["mfma_planes_issued"] = int(info.mfma_planes)
        if form == "hybrid" and info.mfma_planes == 0:
            config["mfma_note"] = ("the tuner measured every level faster by CSR pulls on this graph, so no "
                                   "level ran as an MFMA product in the timed steps")
        if info.mfma_fwd_rows:
            config["mfma_fwd_rows"] = int(info.mfma_fwd_rows)
    if form == "many":
        config["unit_sources"] = int(info.batch)
        config["tune_source"] = ["default", "measured", "cached"][info.tune_source]
    if getattr(wl["graph"], "weight", None) is not None and form == "plain":
        config["bucket_width"] = 1
        config["bucket_note"] = (
            "Delta = 1 (one bucket per distance value, Dial order) is a reading, not a tuned value: counts "
            "sum over predecessors at exactly d(v) - w(u,v), so a wider bucket still needs one phase per "
            "distinct distance and only adds re-relaxations, and the sweep is bound by random sector "
            "reads of the distance arrays that every re-relaxation adds to")
    out = {
        "metric": METRIC if args.workload == "rmat16" else f"BC TEPS (sources·m/s) on {args.workload}",
        "value": work / dt,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[form],
        "data": "synthetic",
        "config": config,
        "tuned_batch_width": free,
        "compare": compare,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kern.items()},
        "time_outside_kernels_frac": max(0.0, 1.0 - sum(v[0] for v in kern.values()) / args.steps / (dt * 1e3)),
        "step_ms": main_step_ms,
        "accuracy": accuracy,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.workload == "rmat16" and "plain" in compare:
        # the headline ratio: batched mixed-precision form over the plain FP64 form
        out["plain_fp64"] = compare["plain"]
        out["batched_vs_plain"] = compare["plain"]["ms_per_step"] / (dt * 1e3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
