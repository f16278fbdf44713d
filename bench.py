#!/usr/bin/env python3
"""Benchmark: speculative graph coloring on one MI355X.

Default workload (d1): a step colors the distance-1 workload of the paper's
on-node hot path once: the 3D 27-point stencil mesh 128^3 (2,097,152
vertices, 53,645,816 directed edges; a PDE mesh like the paper's hexahedral
and SuiteSparse PDE graphs) and the R-MAT scale-22 edge-factor-16 graph (a
power-law graph like the paper's kron_g500 and social networks), each with
color_d1 through the C-ABI.  Inputs are generated (seeded), uploaded and
resident in HBM before timing.

    value  = (nnz_mesh + nnz_rmat) / seconds per step   [edges colored / s]
    d2pd2: the same measurement of the D2 + PD2 workload (--workload d2pd2),
           timed separately after the D1 steps, with its own roofline and
           CPU baseline
    stream_copy: a 1 GiB device copy's GB/s, the practical HBM ceiling
    recolor_degrees: the R-MAT leg colored with the recolorDegrees key
           (Section 3.3) beside the hash key's colors
    cpu_baseline_all_cores: the oracle built with OpenMP, every core
    roofline: the dominant kernel's algorithmic bytes / its HIP-event time;
              traffic: HBM bytes per launch from rocprofv3 FETCH_SIZE and
              WRITE_SIZE runs (profiles/pmc_traffic.json, taken on the same
              library sources, scaled by a plain copy's counters), else null.
    kernels: per timed round kernel, its launches per step, HIP-event time
             per launch, algorithmic bytes and counter bytes per launch
    hbm_counter_rate: the counter bytes of every timed round kernel over
             their summed time (the coloring's %HBM), while the counter
             summary matches the library sources, else null
    cpu_baseline: the CPU oracle on a bounded sample of the same workload.

Other workloads (one JSON line each, same keys):
    --workload batch   a seeded stream of mixed D1/D2/PD2 jobs: color_batch
                       (one persistent launch) against one single-graph call
                       per job; value = graphs/s of the batched form
    --workload serve   the same stream through the continuous-batching
                       server with Poisson arrivals; reports p50/p99 latency
    --workload d2pd2   D2 on the 7-point stencil 96^3 and PD2 on the
                       4,000,000 x 1,000,000 power-law pattern
    --workload ghost   one rank's ghost-layer step (color_d1_ghost) on part 0
                       of a 16-way hash partition of R-MAT scale 24, with 1
                       and 2 ghost layers, fixed ghosts and tentative ghost
                       recoloring, plus property checks
    --workload dist    Algorithm 2 over all 16 ranks of that partition on one
                       GPU (color_d1_distributed)
    --workload ghost2  the distance-2 step on a slab of the 7-point mesh 96^3
                       and the partial distance-2 step on part 0 of the PD2
                       pattern (color_d2_ghost, color_pd2_ghost)

Profiling helpers (no GPU):
    --summarize-pmc FETCH_DIR WRITE_DIR   turns two rocprofv3 --pmc runs
                       (FETCH_SIZE, WRITE_SIZE) of `bench.py --copy-calibration`
                       into profiles/pmc_traffic.json
    --call-rate TRACE_DIR STEPS   %HBM of whole calls (every dispatch): the
                       committed counter summary over the kernel time of one
                       step of a rocprofv3 --kernel-trace run of STEPS steps

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s
def traffic_file(workload):
    """Committed counter summary of a workload's kernels (d1: pmc_traffic.json)."""
    name = "pmc_traffic.json" if workload == "d1" else f"pmc_traffic_{workload}.json"
    return os.path.join(ROOT, "profiles", name)
COPY_BYTES = 1 << 30    # the calibration copy: 1 GiB read + 1 GiB written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def d1_kernel_bytes(st):
    """Algorithmic bytes of the pull engine's D1 color kernel and detect kernel
    over a call.  Per worklist vertex: worklist id, two row offsets, the
    static work value / T[v], and one 4-byte write (T[v], or C[v] / the next
    worklist slot); per adjacency entry: the neighbour id and the neighbour's
    color."""
    color = 20 * st.vertex_visits + 8 * st.edge_visits
    detect = 20 * st.vertex_visits + 8 * st.edge_visits
    return color, detect


def pull_two_hop_bytes(st, avg_deg):
    """Pull engine, D2/PD2: per worklist vertex 20 bytes; per first-hop entry
    its id and the two row offsets of its hop-2 row (12 bytes); per hop-2
    entry its id and color (8 bytes).  edge_visits counts first-hop plus
    hop-2 entries; the first-hop share is estimated as avg_deg per visit."""
    e1 = min(st.edge_visits, int(st.vertex_visits * avg_deg))
    e2 = st.edge_visits - e1
    b = 20 * st.vertex_visits + 12 * e1 + 8 * e2
    return b, b


def make_d1_workload():
    import graphgen as gg
    t = time.time()
    mesh = gg.stencil((128, 128, 128), 27)
    log(f"[bench] mesh 27pt 128^3: n={mesh.n} nnz={mesh.nnz} ({time.time() - t:.1f}s)")
    t = time.time()
    rm = gg.rmat(22, 16, seed=1)
    log(f"[bench] rmat s22 ef16: n={rm.n} nnz={rm.nnz} maxdeg={int(rm.degrees().max())} ({time.time() - t:.1f}s)")
    return [("stencil27_128", mesh), ("rmat22_ef16", rm)]


def cpu_baseline(sample, omp=False):
    """The oracle on the sample graphs: plain single-threaded C, or (omp) the
    same source built with OpenMP on the per-vertex loops of each round, on
    every core the process may use."""
    import oracle
    oracle.build(omp=omp)
    tot_e, tot_t = 0, 0.0
    for name, g in sample:
        t = time.perf_counter()
        r = oracle.color_d1(g, seed=1, omp=omp)
        dt = time.perf_counter() - t
        log(f"[bench] cpu oracle{' (all cores)' if omp else ''} {name}: {dt:.2f}s colors={r.num_colors} "
            f"rounds={r.rounds}")
        tot_e += g.nnz
        tot_t += dt
    return tot_e / tot_t, tot_t


def host_cpu():
    """The host's CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def stream_copy(torch, dev, reps=5):
    """STREAM-copy ceiling of this GPU: a 1 GiB device-to-device copy (1 GiB
    read + 1 GiB written), best of `reps`, timed with events on the current
    stream."""
    a = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    gbs = 2 * COPY_BYTES / (best / 1e3) / 1e9
    log(f"[bench] stream copy: {gbs:.0f} GB/s ({best:.3f} ms for 2 GiB moved)")
    return {"gb_per_s": round(gbs, 1), "bytes_moved": 2 * COPY_BYTES, "ms": round(best, 4),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def load_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    the same workload, if it was taken on the current library sources."""
    try:
        from paper_2107_00075_amd.build import source_hash
        with open(traffic_file(workload)) as f:
            t = json.load(f)
        if t.get("source_hash") != source_hash() or t.get("workload") != workload:
            return None
        k = t["kernels"].get(kernel)
        return None if k is None else int(k["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def counter_rate(kern, workload):
    """Counter-measured HBM bytes (FETCH_SIZE + WRITE_SIZE from the committed
    summary) of all timed round kernels, summed over their launches, over
    their summed HIP-event time: the whole coloring's %HBM.  None unless the
    summary covers every one of them on the current sources."""
    total_b = total_ns = 0
    for kn, (b_alg, ns, nl) in kern.items():
        t = load_traffic(kn, workload)
        if t is None:
            return None
        total_b += t * nl
        total_ns += ns
    if total_ns == 0:
        return None
    gbs = total_b / total_ns
    return {"bytes": int(total_b), "kernel_ms": round(total_ns / 1e6, 3), "gb_per_s": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "kernels": sorted(kern), "note": "round kernels only (setup and list building excluded)"}


def copy_calibration(torch, dev):
    """One plain device copy of COPY_BYTES (its counters scale FETCH_SIZE and
    WRITE_SIZE to bytes)."""
    a = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def kernel_rows(gc, st, names, color_bytes, detect_bytes):
    """(kernel, algorithmic bytes, HIP-event ns, launches) of one call's round
    kernels; the incremental engine's cooperative tail kernel (all rounds once
    the worklist is small, in one launch) is a kernel of its own."""
    rows = [(names[0], color_bytes, st.color_kernel_ns, st.color_launches),
            (names[1], detect_bytes, st.detect_kernel_ns, st.detect_launches)]
    if st.tail_rounds:
        rows.append(("inc_tail_kernel", st.tail_bytes, st.tail_kernel_ns, 1))
    return rows


def bench_d1(args, torch, gc, dev):
    work = make_d1_workload()
    graphs = []
    for name, g in work:
        graphs.append((name, g, torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                       torch.empty(g.n, dtype=torch.int32, device=dev)))
    torch.cuda.synchronize()
    if args.copy_calibration:
        copy_calibration(torch, dev)
    params = gc.Params(flags=gc.COLOR_FLAG_KERNEL_TIMING)

    def step():
        out = []
        for name, g, rp, ci, colors in graphs:
            _, st = gc.color_d1(rp, ci, seed=1, out=colors, params=params)
            out.append(st)
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per_step = []
    stats = []
    t_all = time.perf_counter()
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(step())
        torch.cuda.synchronize()
        per_step.append(time.perf_counter() - t0)
        log(f"[bench] step {i}: {per_step[-1] * 1e3:.2f} ms")
    t_all = time.perf_counter() - t_all
    ms = 1e3 * t_all / args.steps
    nnz_total = sum(g.nnz for _, g, *_ in graphs)
    value = nnz_total / (t_all / args.steps)

    # roofline of the dominant kernel over the timed steps.  Pull engine: the
    # algorithmic bytes follow from the visit counters (d1_kernel_bytes);
    # incremental engine: its kernels count their own algorithmic bytes.
    kern = {}
    per_graph = {}
    for s_list in stats:
        for (name, g, *_), st in zip(graphs, s_list):
            if st.engine == gc.ENGINE_INCREMENTAL:
                names = ("inc_color_kernel", "inc_detect_kernel")
                cb, db = st.color_bytes, st.detect_bytes
            else:
                names = ("color_round_kernel<D1>", "detect_round_kernel<D1>")
                cb, db = d1_kernel_bytes(st)
            for kname, byts, ns, nl in kernel_rows(gc, st, names, cb, db):
                acc = kern.setdefault(kname, [0, 0, 0])
                acc[0] += byts
                acc[1] += ns
                acc[2] += nl
            pg = per_graph.setdefault(name, {"nnz": g.nnz, "n": g.n, "colors": st.num_colors,
                                             "rounds": st.rounds, "edge_visits": st.edge_visits,
                                             "vertex_visits": st.vertex_visits, "kernel_ms": 0.0,
                                             "engine": {1: "pull", 2: "incremental"}.get(st.engine, "?"),
                                             "list_visits": st.list_visits})
            pg["kernel_ms"] += (st.color_kernel_ns + st.detect_kernel_ns + st.tail_kernel_ns) / 1e6 / args.steps
            pg["tail_rounds"] = st.tail_rounds
    dom = max(kern, key=lambda k: kern[k][1])
    b, ns, launches = kern[dom]
    achieved = b / ns if ns else 0.0   # bytes per ns == GB/s
    traffic = load_traffic(dom, "d1")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "avg_launch_us": round(ns / max(launches, 1) / 1e3, 3),
                "alg_bytes_per_launch": int(b / max(launches, 1)),
                "launches_per_step": launches // max(args.steps, 1)}
    # every timed round kernel: algorithmic bytes and HIP-event time per launch
    kernels = {kn: {"launches_per_step": kv[2] // max(args.steps, 1),
                    "avg_launch_us": round(kv[1] / max(kv[2], 1) / 1e3, 3),
                    "alg_bytes_per_launch": int(kv[0] / max(kv[2], 1)),
                    "achieved_gb_per_s": round(kv[0] / kv[1], 1) if kv[1] else None,
                    "counter_bytes_per_launch": load_traffic(kn, "d1")}
               for kn, kv in kern.items()}
    hbm_rate = counter_rate(kern, "d1")
    for name, pg in per_graph.items():
        pg["edges_per_s_kernels_only"] = round(pg["nnz"] / (pg["kernel_ms"] / 1e3), 1) if pg["kernel_ms"] else None

    # recolorDegrees (Section 3.3) on the R-MAT leg: colors and time against
    # the hash key of the timed steps
    rd = copy = None
    if not args.no_extras:
        name, g, rp, ci, colors = graphs[1]
        rd_params = gc.Params(flags=gc.COLOR_FLAG_RECOLOR_DEGREES)
        gc.color_d1(rp, ci, seed=1, out=colors, params=rd_params)
        rd_ms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = gc.color_d1(rp, ci, seed=1, out=colors, params=rd_params)
            torch.cuda.synchronize()
            rd_ms.append((time.perf_counter() - t0) * 1e3)
        hash_st = stats[-1][1]
        rd = {"graph": name, "colors": st.num_colors, "rounds": st.rounds, "ms": round(sorted(rd_ms)[1], 3),
              "hash_key_colors": hash_st.num_colors, "hash_key_rounds": hash_st.rounds,
              "hash_key_kernel_ms": round(per_graph[name]["kernel_ms"], 3)}
        log(f"[bench] recolorDegrees on {name}: {st.num_colors} colors in {rd['ms']:.1f} ms "
            f"(hash key: {hash_st.num_colors} colors)")
        copy = stream_copy(torch, dev)

    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        import graphgen as gg
        import oracle
        sample = [("stencil27_128", work[0][1]), ("rmat20_ef16", gg.rmat(20, 16, seed=1))]
        what = "27-pt stencil 128^3 (full) + R-MAT scale 20 ef16 (1/4 of the R-MAT leg)"
        v, secs = cpu_baseline(sample)
        cpu = {"value": round(v, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"{what}, single-threaded C oracle, {secs:.1f}s"}
        v, secs = cpu_baseline(sample, omp=True)
        cpu_all = {"value": round(v, 1), "unit": "edges/s", "cores": oracle.threads(omp=True), "kind": "oracle",
                   "sample": f"{what}, the same C oracle built with OpenMP on the per-vertex loops of each "
                             f"round, {secs:.1f}s", "host": host_cpu()}

    sub = None
    if not args.no_d2pd2:
        r = bench_d2pd2(args, torch, gc, dev)
        sub = {k: r[k] for k in ("metric", "value", "unit", "ms_per_step", "config", "roofline", "hbm_counter_rate",
                                 "cpu_baseline")}

    return {
        "metric": "edges colored/s (D1)",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "D1 coloring: 27-pt stencil 128^3 + R-MAT s22 ef16 (a,b,c)=(.57,.19,.19), "
                               "symmetrized, deduplicated; int32 CSR; seed 1",
                   "graphs": per_graph},
        "roofline": roofline,
        "kernels": kernels,
        "hbm_counter_rate": hbm_rate,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "stream_copy": copy,
        "recolor_degrees": rd,
        "d2pd2": sub,
    }


# ---------------------------------------------------------------------------
# distance-2 and partial distance-2
# ---------------------------------------------------------------------------

def bench_d2pd2(args, torch, gc, dev):
    """D2 on the 7-point stencil 96^3 and PD2 on the 4,000,000 x 1,000,000
    power-law pattern (8 columns per row, tail exponent 2.1), one step = both."""
    import graphgen as gg
    t = time.time()
    g = gg.stencil((96, 96, 96), 7)
    b = gg.bipartite_powerlaw(4_000_000, 1_000_000, 8, 2.1, seed=1)
    log(f"[bench] 7pt 96^3: n={g.n} nnz={g.nnz}; PD2 {b.n_rows}x{b.n_cols} nnz={b.nnz} ({time.time() - t:.1f}s)")
    d = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    grp, gci = d(g.row_ptr), d(g.col)
    brp, bci, bcp, bri = d(b.row_ptr), d(b.col_idx), d(b.col_ptr), d(b.row_idx)
    out_d2 = torch.empty(g.n, dtype=torch.int32, device=dev)
    out_pd2 = torch.empty(b.n_cols, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    if args.copy_calibration:
        copy_calibration(torch, dev)
    params = gc.Params(flags=gc.COLOR_FLAG_KERNEL_TIMING)

    def step():
        _, s1 = gc.color_d2(grp, gci, seed=1, out=out_d2, params=params)
        _, s2 = gc.color_pd2(brp, bci, bcp, bri, seed=1, out=out_pd2, params=params)
        return s1, s2

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    times, stats = [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(step())
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[bench] step {i}: {times[-1] * 1e3:.1f} ms")
    tm = sum(times) / len(times)
    kern, graphs = {}, {}
    for s1, s2 in stats:
        for name, st, nnz, deg, mode in (("stencil7_96_d2", s1, g.nnz, g.nnz / g.n, "D2"),
                                         ("pd2_4m_1m", s2, b.nnz, b.nnz / b.n_cols, "PD2")):
            if st.engine == gc.ENGINE_INCREMENTAL:
                names, (cb, db) = ("inc_color_kernel", "inc_detect_kernel"), (st.color_bytes, st.detect_bytes)
            else:
                names = (f"color_round_kernel<{mode}>", f"detect_round_kernel<{mode}>")
                cb, db = pull_two_hop_bytes(st, deg)
            for kname, byts, ns, nl in kernel_rows(gc, st, names, cb, db):
                acc = kern.setdefault(kname, [0, 0, 0])
                acc[0] += byts
                acc[1] += ns
                acc[2] += nl
            pg = graphs.setdefault(name, {"nnz": nnz, "colors": st.num_colors, "rounds": st.rounds,
                                          "edge_visits": st.edge_visits, "vertex_visits": st.vertex_visits,
                                          "engine": {1: "pull", 2: "incremental"}.get(st.engine, "?"),
                                          "kernel_ms": 0.0})
            pg["kernel_ms"] += (st.color_kernel_ns + st.detect_kernel_ns + st.tail_kernel_ns) / 1e6 / args.steps
            pg["tail_rounds"] = st.tail_rounds
    dom = max(kern, key=lambda k: kern[k][1])
    byts, ns, launches = kern[dom]
    achieved = byts / ns if ns else 0.0
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on D2 96^3 (full) and on the PD2 pattern at 1/10 of its rows and columns
        import oracle
        oracle.build()
        small = gg.bipartite_powerlaw(200_000, 50_000, 8, 2.1, seed=1)
        t0 = time.perf_counter()
        r1 = oracle.color_d2(g, seed=1)
        t1 = time.perf_counter()
        r2 = oracle.color_pd2(small, seed=1)
        t2 = time.perf_counter()
        log(f"[bench] cpu oracle D2 96^3: {t1 - t0:.1f}s ({r1.num_colors} colors); "
            f"PD2 200k x 50k: {t2 - t1:.1f}s ({r2.num_colors} colors)")
        cpu = {"value": round((g.nnz + small.nnz) / (t2 - t0), 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"D2 on 7-pt 96^3 (full) + PD2 on the 200,000 x 50,000 pattern of the same recipe "
                         f"(1/20 of the PD2 leg), single-threaded C oracle, {t2 - t0:.1f}s"}
    return {
        "metric": "edges colored/s (D2 + PD2)",
        "value": round((g.nnz + b.nnz) / tm, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tm * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "D2 on 7-pt stencil 96^3 + PD2 (columns) on 4,000,000 x 1,000,000 power-law pattern, "
                               "8 columns per row, gamma 2.1; seed 1", "graphs": graphs},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(dom, "d2pd2"),
                     "avg_launch_us": round(ns / max(launches, 1) / 1e3, 3),
                     "alg_bytes_per_launch": int(byts / max(launches, 1))},
        "hbm_counter_rate": counter_rate(kern, "d2pd2"),
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------------------
# batched and served forms
# ---------------------------------------------------------------------------

def _stream(args):
    import graphgen as gg
    t = time.time()
    specs = gg.job_stream(args.jobs, seed=args.stream_seed, n_min=1_000, n_max=args.n_max)
    kinds = [s.kind for s in specs]
    log(f"[bench] {len(specs)} jobs (D1 {kinds.count(1)}, D2 {kinds.count(2)}, PD2 {kinds.count(3)}), "
        f"sum n {sum(s.graph.n for s in specs)}, sum nnz {sum(s.graph.nnz for s in specs)} "
        f"({time.time() - t:.1f}s)")
    return specs


def _nnz_of(s):
    return s.pattern.nnz if s.kind == 3 else s.graph.nnz


def bench_batch(args, torch, gc, dev):
    specs = _stream(args)

    def d(a):
        return torch.from_numpy(a).to(dev)

    jobs = []
    for s in specs:
        if s.kind == 3:
            b = s.pattern
            jobs.append({"kind": 3, "row_ptr": d(b.row_ptr), "col_idx": d(b.col_idx), "col_ptr": d(b.col_ptr),
                         "row_idx": d(b.row_idx), "seed": s.seed})
        else:
            jobs.append({"kind": s.kind, "row_ptr": d(s.graph.row_ptr), "col_idx": d(s.graph.col), "seed": s.seed})
        n = (jobs[-1]["col_ptr"] if s.kind == 3 else jobs[-1]["row_ptr"]).numel() - 1
        jobs[-1]["out"] = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    plain_out = [torch.empty_like(j["out"]) for j in jobs]
    torch.cuda.synchronize()

    def plain():
        for j, o in zip(jobs, plain_out):
            if j["kind"] == 3:
                gc.color_pd2(j["row_ptr"], j["col_idx"], j["col_ptr"], j["row_idx"], seed=j["seed"], out=o)
            elif j["kind"] == 2:
                gc.color_d2(j["row_ptr"], j["col_idx"], seed=j["seed"], out=o)
            else:
                gc.color_d1(j["row_ptr"], j["col_idx"], seed=j["seed"], out=o)

    def batched():
        return gc.color_batch(jobs)[1]

    for i in range(args.warmup):
        t0 = time.perf_counter()
        plain()
        torch.cuda.synchronize()
        log(f"[bench] warm-up {i}: plain {1e3 * (time.perf_counter() - t0):.1f} ms")
        t0 = time.perf_counter()
        batched()
        torch.cuda.synchronize()
        log(f"[bench] warm-up {i}: batched {1e3 * (time.perf_counter() - t0):.1f} ms")
    t_plain, t_batch = [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain()
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        st = batched()
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - t0)
        log(f"[bench] step {i}: plain {t_plain[-1] * 1e3:.1f} ms, batched {t_batch[-1] * 1e3:.1f} ms")
    same = all(torch.equal(j["out"], o) for j, o in zip(jobs, plain_out))
    tb = sum(t_batch) / len(t_batch)
    tp = sum(t_plain) / len(t_plain)
    nnz = sum(_nnz_of(s) for s in specs)
    return {
        "metric": "graphs colored/s (batched, mixed D1/D2/PD2)",
        "value": round(len(specs) / tb, 1),
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tb * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} jobs, n log-uniform [1e3, {args.n_max:g}], ER/stencil/R-MAT thirds, "
                               f"D1/D2/PD2 70/20/10 (D2, PD2 on ER and stencil), seed {args.stream_seed}",
                   "sum_nnz": nnz, "rounds_max": max(x.rounds for x in st)},
        "plain_per_graph": {"ms_per_step": round(tp * 1e3, 3), "graphs_per_s": round(len(specs) / tp, 1)},
        "speedup_vs_plain": round(tp / tb, 3),
        "edges_per_s_batched": round(nnz / tb, 1),
        "identical_colorings": bool(same),
        "roofline": None,
        "cpu_baseline": None,
    }


def bench_serve(args, torch, gc, dev):
    import numpy as np
    specs = _stream(args)
    budget = int(args.serve_budget_gib * (1 << 30))

    def submit(srv, s):
        if s.kind == 3:
            b = s.pattern
            return srv.submit(3, b.row_ptr, b.col_idx, b.col_ptr, b.row_idx, seed=s.seed)[0]
        return srv.submit(s.kind, s.graph.row_ptr, s.graph.col, seed=s.seed)[0]

    def run(rate, keep=None):
        """Open loop at `rate` jobs/s (None: all at t=0).  Returns latencies (s) and makespan.
        keep: a list that receives every job's host colors, in stream order."""
        rng = np.random.default_rng(123)
        gaps = rng.exponential(1.0 / rate, len(specs)) if rate else np.zeros(len(specs))
        arrive = np.cumsum(gaps)
        srv = gc.ColorServer(budget, max_slots=args.slots)
        lat, pending = [], {}
        index = {}
        nxt = 0
        t0 = time.perf_counter()
        t_log = t0
        try:
            while nxt < len(specs) or pending:
                now = time.perf_counter() - t0
                if now + t0 - t_log > 10.0:
                    t_log = now + t0
                    log(f"[bench] serve: {len(lat)} of {len(specs)} jobs done after {now:.1f} s")
                while nxt < len(specs) and arrive[nxt] <= now:
                    jid = submit(srv, specs[nxt])
                    pending[jid] = arrive[nxt]
                    index[jid] = nxt
                    nxt += 1
                for jid in list(pending):
                    r = srv.poll(jid)
                    if r is not None:
                        lat.append(time.perf_counter() - t0 - pending.pop(jid))
                        if keep is not None:
                            keep[index[jid]] = r[0]
        finally:
            srv.close()
        return np.array(lat), time.perf_counter() - t0

    served = [None] * len(specs)
    _, span0 = run(None, keep=served)  # warm-up (library and page-in); its colorings are checked below
    log(f"[bench] serve warm-up: {span0:.2f} s")
    # the plain single-graph call of each job's kind from the same host
    # arrays (copy in, color, copy the colors out: the work a served job
    # includes), timed as one pass; every served coloring is compared with it
    def plain_from_host(s):
        if s.kind == 3:
            b = s.pattern
            ref, _ = gc.color_pd2(*(torch.from_numpy(a).to(dev) for a in (b.row_ptr, b.col_idx, b.col_ptr,
                                                                          b.row_idx)), seed=s.seed)
        else:
            fn = gc.color_d2 if s.kind == 2 else gc.color_d1
            ref, _ = fn(torch.from_numpy(s.graph.row_ptr).to(dev), torch.from_numpy(s.graph.col).to(dev),
                        seed=s.seed)
        return ref.cpu().numpy()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_colors = [plain_from_host(s) for s in specs]
    torch.cuda.synchronize()
    t_plain_host = time.perf_counter() - t0
    log(f"[bench] plain calls from host arrays: {len(specs) / t_plain_host:.1f} graphs/s")
    same = all(got is not None and np.array_equal(ref, np.asarray(got)) for ref, got in zip(plain_colors, served))
    del plain_colors
    log(f"[bench] served colorings identical to the plain calls: {same}")
    lat_closed, span = run(None)
    sat = len(specs) / span
    log(f"[bench] serve closed-loop: {sat:.1f} graphs/s, p50 {np.percentile(lat_closed, 50) * 1e3:.1f} ms")
    loads = {}
    for f in (0.5, 0.8, 1.2):
        lat, span_f = run(f * sat)
        loads[str(f)] = {"rate_graphs_per_s": round(f * sat, 1),
                         "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                         "throughput_graphs_per_s": round(len(specs) / span_f, 1)}
        log(f"[bench] serve {f}x: {loads[str(f)]}")
    return {
        "metric": "p99 latency (served, 0.8x saturation)",
        "value": loads["0.8"]["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(span * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} jobs as the batch workload (n log-uniform [1e3, {args.n_max:g}]), "
                               f"Poisson arrivals at 0.5/0.8/1.2x the "
                               f"closed-loop rate; server budget {args.serve_budget_gib} GiB, {args.slots} slots",
                   "closed_loop_graphs_per_s": round(sat, 1),
                   "closed_loop_p50_ms": round(float(np.percentile(lat_closed, 50)) * 1e3, 3),
                   "loads": loads},
        "identical_colorings": bool(same),
        "plain_from_host": {"graphs_per_s": round(len(specs) / t_plain_host, 1),
                            "note": "single-graph call per job with its host arrays copied in and colors out"},
        "closed_loop_speedup_vs_plain_from_host": round(sat * t_plain_host / len(specs), 3),
        "roofline": None,
        "cpu_baseline": None,
    }


# ---------------------------------------------------------------------------
# ghost-layer step on one part of a partitioned graph
# ---------------------------------------------------------------------------

def _timed(torch, args, fn):
    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = fn()
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t0) / args.steps


def bench_ghost(args, torch, gc, dev):
    """One rank's step (color_d1_ghost) on part 0 of a 16-way hash partition
    of R-MAT scale `--ghost-scale`, with 1 and 2 ghost layers, with the ghosts'
    colors fixed and with tentative ghost recoloring (Section 3.2 / 3.4).
    Checks properties that hold at any size: owned colors proper among owned
    vertices, every owned-ghost pair still equal after the step has its ghost
    flagged as a remote loser, and (fixed ghosts) the 2-layer result equal to
    the 1-layer one."""
    import numpy as np

    import graphgen as gg
    t = time.time()
    g = gg.rmat(args.ghost_scale, 16, seed=1, progress=lambda m: log(f"[bench] {m} ({time.time() - t:.0f}s)"))
    delta = int(g.degrees().max())
    log(f"[bench] rmat s{args.ghost_scale}: n={g.n} nnz={g.nnz} maxdeg={delta} ({time.time() - t:.1f}s)")
    owner = gg.hash_partition(g.n, 16, seed=7)
    gcol = gg.ghost_colors_uniform(g.n, delta, seed=11)
    res, rec = {}, {}
    kern = {}
    for layers in (1, 2):
        t = time.time()
        log(f"[bench] building part 0 with {layers} ghost layer(s)")
        lg = gg.ghost_local_graph(g, owner, 0, layers, gcol, sort_rows=False)
        log(f"[bench] part 0, {layers} layer(s): owned {lg.n_owned}, ghosts {lg.n_ghost} (G1 {lg.n_g1}), "
            f"local nnz {lg.nnz} ({time.time() - t:.1f}s)")
        rp, ci, gid, gco = (torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                            for a in (lg.row_ptr, lg.col, lg.gid, lg.ghost_colors))
        out = torch.empty(lg.n_owned, dtype=torch.int32, device=dev)
        timing = gc.Params(flags=gc.COLOR_FLAG_KERNEL_TIMING)
        (colors, rl, st), dt = _timed(torch, args, lambda: gc.color_d1_ghost(
            lg.n_owned, lg.n_ghost, layers, lg.n_g1, rp, ci, gid, gco, seed=1, out=out, params=timing))
        colors, rl = colors.cpu().numpy(), rl.cpu().numpy()
        owned_nnz = int(lg.row_ptr[lg.n_owned])
        res[layers] = {"colors": colors, "rl": rl, "st": st, "ms": dt * 1e3, "lg": lg, "owned_nnz": owned_nnz}
        log(f"[bench] {layers} layer(s): {dt * 1e3:.2f} ms, colors {st.num_colors}, rounds {st.rounds}, "
            f"conflicts {st.boundary_conflicts}, remote losers {st.remote_losers}, engine {st.engine}")
        if layers == 1:
            names = ("inc_color_kernel", "inc_detect_kernel") if st.engine == gc.ENGINE_INCREMENTAL else \
                ("color_round_kernel<D1>", "detect_round_kernel<D1>")
            cb, db = (st.color_bytes, st.detect_bytes) if st.engine == gc.ENGINE_INCREMENTAL else d1_kernel_bytes(st)
            for kname, byts, ns, nl in kernel_rows(gc, st, names, cb, db):
                kern[kname] = (byts, ns, nl)
        grp = gc.Params(flags=gc.COLOR_FLAG_GHOST_RECOLOR)
        (c2, rl2, st2), dt2 = _timed(torch, args, lambda: gc.color_d1_ghost(
            lg.n_owned, lg.n_ghost, layers, lg.n_g1, rp, ci, gid, gco, seed=1, out=out, params=grp))
        rec[layers] = {"ms": round(dt2 * 1e3, 3), "colors": st2.num_colors, "rounds": st2.rounds,
                       "boundary_conflicts": st2.boundary_conflicts, "remote_losers": st2.remote_losers,
                       "differs_from_fixed_ghosts": int(np.count_nonzero(c2.cpu().numpy() != colors))}
        log(f"[bench] {layers} layer(s), tentative ghost recoloring: {dt2 * 1e3:.2f} ms, {st2.num_colors} colors")
        del rp, ci, gid, gco
    # properties on the 1-layer local graph
    lg = res[1]["lg"]
    colors, rl = res[1]["colors"], res[1]["rl"]
    no = lg.n_owned
    src = np.repeat(np.arange(no), np.diff(lg.row_ptr[:no + 1]))
    dst = lg.col[:lg.row_ptr[no]]
    inner = dst < no
    proper = bool(np.all(colors[src[inner]] != colors[dst[inner]])) and bool(colors.min() >= 1)
    gdst = dst[~inner] - no
    eq = colors[src[~inner]] == lg.ghost_colors[gdst]
    flagged = bool(np.all(rl[gdst[eq]] == 1))
    same_layers = bool(np.array_equal(res[1]["colors"], res[2]["colors"]) and
                       np.array_equal(res[1]["rl"], res[2]["rl"][:res[1]["rl"].size]))
    st1 = res[1]["st"]
    roofline = None
    if kern:
        dom = max(kern, key=lambda k: kern[k][1])
        b_, ns, nl = kern[dom]
        ach = b_ / ns if ns else 0.0
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                    "avg_launch_us": round(ns / max(nl, 1) / 1e3, 3), "alg_bytes_per_launch": int(b_ / max(nl, 1))}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        t0 = time.perf_counter()
        r = oracle.color_d1_ghost(lg, seed=1)
        secs = time.perf_counter() - t0
        assert np.array_equal(r.colors, colors), "oracle and GPU differ on part 0"
        cpu = {"value": round(res[1]["owned_nnz"] / secs, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"the same step (part 0, 1 layer), single-threaded C oracle, {secs:.1f}s"}
    return {
        "metric": "edges colored/s (D1 ghost-layer step, part 0 of 16)",
        "value": round(res[1]["owned_nnz"] / (res[1]["ms"] / 1e3), 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res[1]["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT s{args.ghost_scale} ef16 seed 1, 16-way hash partition, part 0, ghost colors "
                               f"uniform in [1, maxdeg+1]; 1 and 2 ghost layers",
                   "layers": {str(k): {"ms": round(v["ms"], 3), "owned": v["lg"].n_owned,
                                       "ghosts": v["lg"].n_ghost, "local_nnz": v["lg"].nnz,
                                       "owned_row_nnz": v["owned_nnz"], "colors": v["st"].num_colors,
                                       "rounds": v["st"].rounds,
                                       "boundary_conflicts": v["st"].boundary_conflicts,
                                       "remote_losers": v["st"].remote_losers} for k, v in res.items()},
                   "tentative_ghost_recoloring": {str(k): v for k, v in rec.items()},
                   "checks": {"owned_proper": proper, "equal_pairs_flagged": flagged,
                              "two_layers_equal_one": same_layers}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "boundary_conflicts": st1.boundary_conflicts,
    }


def bench_dist(args, torch, gc, dev):
    """Algorithm 2 over 16 ranks on one GPU (color_d1_distributed): R-MAT
    scale `--ghost-scale` split 16 ways by hash, every rank's local graph
    with one ghost layer resident; one step = the whole distributed coloring
    (initial colorings, exchanges, detections, recolorings until no
    conflict), with the hash key, recolorDegrees and tentative ghost
    recoloring."""
    import numpy as np

    import graphgen as gg
    t = time.time()
    g = gg.rmat(args.ghost_scale, 16, seed=1, progress=lambda m: log(f"[bench] {m} ({time.time() - t:.0f}s)"))
    log(f"[bench] rmat s{args.ghost_scale}: n={g.n} nnz={g.nnz} ({time.time() - t:.1f}s)")
    owner = gg.hash_partition(g.n, 16, seed=7)
    zeros = np.zeros(g.n, np.int32)
    deg = g.degrees()
    parts, locs = [], []
    for p in range(16):
        lg = gg.ghost_local_graph(g, owner, p, 1, zeros, sort_rows=False)
        locs.append(lg)
    homes = gg.ghost_homes(locs)
    for lg, (o, i) in zip(locs, homes):
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)  # noqa: E731
        parts.append(dict(n_owned=lg.n_owned, n_ghost=lg.n_ghost, layers=1, n_g1=lg.n_g1, row_ptr=d(lg.row_ptr),
                          col_idx=d(lg.col), gid=d(lg.gid), ghost_owner=d(o), ghost_index=d(i),
                          ghost_degree=d(deg[lg.gid[lg.n_owned:]])))
    log(f"[bench] 16 local graphs resident ({time.time() - t:.1f}s)")
    out = {}
    for name, flags in (("hash_key", 0), ("recolor_degrees", gc.COLOR_FLAG_RECOLOR_DEGREES),
                        ("ghost_recoloring", gc.COLOR_FLAG_GHOST_RECOLOR)):
        few = argparse.Namespace(steps=min(args.steps, 2), warmup=min(args.warmup, 1))
        (cols, st), dt = _timed(torch, few, lambda: gc.color_d1_distributed(parts, seed=1,
                                                                          params=gc.Params(flags=flags)))
        out[name] = {"ms": round(dt * 1e3, 3), "colors": st.num_colors, "detects": st.detects,
                     "iterations": st.iterations, "conflicts": st.conflicts, "exchanged": st.exchanged,
                     "exchanged_bytes": 8 * st.exchanged_total, "rounds_total": st.rounds_total}
        log(f"[bench] Algorithm 2, {name}: {dt * 1e3:.1f} ms, {st.num_colors} colors, {st.detects} detections, "
            f"{8 * st.exchanged_total} bytes exchanged")
        if name == "hash_key":
            C = np.zeros(g.n, np.int32)
            for lg, c in zip(locs, cols):
                C[lg.gid[:lg.n_owned]] = c.cpu().numpy()
            src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
            out[name]["proper"] = bool(np.all(C[src] != C[g.col]))
    rp, ci = torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev)
    (_, st1), dt1 = _timed(torch, args, lambda: gc.color_d1(rp, ci, seed=1))
    one = {"ms": round(dt1 * 1e3, 3), "colors": st1.num_colors, "rounds": st1.rounds}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        small = gg.rmat(19, 16, seed=1)
        ow = gg.hash_partition(small.n, 16, seed=7)
        sl = [gg.ghost_local_graph(small, ow, p, 1, np.zeros(small.n, np.int32)) for p in range(16)]
        t0 = time.perf_counter()
        oracle.color_d1_distributed(sl, seed=1)
        secs = time.perf_counter() - t0
        cpu = {"value": round(small.nnz / secs, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"Algorithm 2 over 16 ranks of R-MAT scale 19 ef16 (1/32 of the graph), single-threaded "
                         f"C oracle per rank step, {secs:.1f}s"}
    base = out["hash_key"]
    return {
        "metric": "edges colored/s (Algorithm 2 over 16 ranks on one GPU)",
        "value": round(g.nnz / (base["ms"] / 1e3), 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": base["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT s{args.ghost_scale} ef16 seed 1 split 16 ways by hash (seed 7), one ghost "
                               f"layer, every rank resident; exchanges by gather kernel",
                   "variants": out, "single_gpu_color_d1": one},
        "roofline": None,
        "cpu_baseline": cpu,
    }


def bench_ghost2(args, torch, gc, dev):
    """One rank's distance-2 step (color_d2_ghost) on a middle slab of the
    7-point mesh 96^3 split into 16 slabs along z, and one rank's partial
    distance-2 step (color_pd2_ghost) on part 0 of the 4,000,000 x 1,000,000
    power-law pattern split 16 ways by column hash; ghost colors uniform in
    [1, 25] (mesh: the distance-2 neighbourhood has 24 members) and [1, 64]."""
    import numpy as np

    import graphgen as gg
    t = time.time()
    dims = (96, 96, 96)
    mesh = gg.stencil(dims, 7)
    lg = gg.ghost_local_graph(mesh, gg.slab_partition(dims, 16), 1, 2,
                              np.random.default_rng(11).integers(1, 26, mesh.n).astype(np.int32))
    b = gg.bipartite_powerlaw(4_000_000, 1_000_000, 8, 2.1, seed=1)
    lp = gg.pd2_local_pattern(b, gg.hash_partition(b.n_cols, 16, seed=7), 0,
                              np.random.default_rng(12).integers(1, 65, b.n_cols).astype(np.int32))
    log(f"[bench] D2 slab: owned {lg.n_owned}, ghosts {lg.n_ghost}; PD2 part 0: owned {lp.n_owned} columns, "
        f"ghosts {lp.n_ghost}, rows {lp.n_rows} ({time.time() - t:.1f}s)")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)  # noqa: E731
    m_args = (lg.n_owned, lg.n_ghost, lg.n_g1, d(lg.row_ptr), d(lg.col), d(lg.gid), d(lg.ghost_colors))
    p_args = (lp.n_owned, lp.n_ghost, lp.n_rows, d(lp.col_ptr), d(lp.row_idx), d(lp.row_ptr), d(lp.col_idx),
              d(lp.gid), d(lp.ghost_colors))
    (c1, r1, s1), dt1 = _timed(torch, args, lambda: gc.color_d2_ghost(*m_args, seed=1))
    (c2, r2, s2), dt2 = _timed(torch, args, lambda: gc.color_pd2_ghost(*p_args, seed=1))
    m_nnz = int(lg.row_ptr[lg.n_owned])
    p_nnz = int(lp.col_ptr[lp.n_owned])
    res = {"d2_mesh_slab": {"ms": round(dt1 * 1e3, 3), "owned": lg.n_owned, "ghosts": lg.n_ghost,
                            "owned_row_nnz": m_nnz, "colors": s1.num_colors, "rounds": s1.rounds,
                            "boundary_conflicts": s1.boundary_conflicts, "remote_losers": s1.remote_losers},
           "pd2_part0": {"ms": round(dt2 * 1e3, 3), "owned": lp.n_owned, "ghosts": lp.n_ghost, "rows": lp.n_rows,
                         "owned_col_nnz": p_nnz, "colors": s2.num_colors, "rounds": s2.rounds,
                         "boundary_conflicts": s2.boundary_conflicts, "remote_losers": s2.remote_losers}}
    log(f"[bench] D2 ghost: {dt1 * 1e3:.2f} ms; PD2 ghost: {dt2 * 1e3:.2f} ms")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        t0 = time.perf_counter()
        ref = oracle.color_d2_ghost(lg, seed=1)
        secs = time.perf_counter() - t0
        assert np.array_equal(ref.colors, c1.cpu().numpy()), "oracle and GPU differ on the mesh slab"
        cpu = {"value": round(m_nnz / secs, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"the D2 mesh-slab step, single-threaded C oracle, {secs:.1f}s"}
    return {
        "metric": "edges colored/s (D2 + PD2 ghost-layer steps)",
        "value": round((m_nnz + p_nnz) / (dt1 + dt2), 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((dt1 + dt2) * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "D2: 7-pt mesh 96^3 in 16 z-slabs, slab 1, 2 ghost layers; PD2: 4,000,000 x "
                               "1,000,000 power-law pattern, 16-way column hash, part 0", "steps": res},
        "roofline": None,
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------------------
# hardware-counter summary (runs on the host, no GPU)
# ---------------------------------------------------------------------------

def _counter_rows(d):
    """Per-dispatch counter values from a rocprofv3 output folder: the CSV
    output (*counter_collection.csv) or the rocpd database (*.db), whose
    `counters_collection` view holds the same rows."""
    rows = []
    for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(fn, newline="") as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        import sqlite3
        for fn in glob.glob(os.path.join(d, "**", "*.db"), recursive=True):
            con = sqlite3.connect(fn)
            for name, counter, value in con.execute(
                    "select kernel_name, counter_name, value from counters_collection"):
                rows.append({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})
            con.close()
    if not rows:
        raise SystemExit(f"no counter rows (*counter_collection.csv or rocpd *.db) under {d}")
    return rows


def _short(name):
    base = name.split("(")[0].replace("void ", "").replace("gcol::", "").strip()
    return base.replace("<1>", "<D1>").replace("<2>", "<D2>").replace("<3>", "<PD2>")


def summarize_pmc(fetch_dir, write_dir, workload, out):
    """KiB per dispatch from FETCH_SIZE / WRITE_SIZE runs -> bytes per launch
    per kernel, scaled so that the calibration copy reads and writes
    COPY_BYTES each."""
    from paper_2107_00075_amd.build import source_hash
    per = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        for r in _counter_rows(d):
            if not r.get("Counter_Name", "").startswith(counter):
                continue
            k = _short(r["Kernel_Name"])
            e = per.setdefault(k, {}).setdefault(counter, [])
            e.append(float(r["Counter_Value"]))
    copy_keys = [k for k in per if "copyBuffer" in k]
    if not copy_keys:
        raise SystemExit("no copy kernel in the runs: profile bench.py --copy-calibration")
    ck = copy_keys[0]
    fetch_copy = max(per[ck]["FETCH_SIZE"]) * 1024.0
    write_copy = max(per[ck]["WRITE_SIZE"]) * 1024.0
    f_scale = COPY_BYTES / fetch_copy
    w_scale = COPY_BYTES / write_copy
    kernels = {}
    for k, v in per.items():
        if "FETCH_SIZE" not in v or "WRITE_SIZE" not in v:
            continue
        fb = sum(v["FETCH_SIZE"]) / len(v["FETCH_SIZE"]) * 1024.0 * f_scale
        wb = sum(v["WRITE_SIZE"]) / len(v["WRITE_SIZE"]) * 1024.0 * w_scale
        kernels[k] = {"dispatches": len(v["FETCH_SIZE"]), "fetch_bytes_per_launch": int(fb),
                      "write_bytes_per_launch": int(wb), "hbm_bytes_per_launch": int(fb + wb)}
    res = {"source_hash": source_hash(), "workload": workload,
           "copy_calibration": {"kernel": ck, "bytes": COPY_BYTES, "fetch_scale": round(f_scale, 4),
                                "write_scale": round(w_scale, 4)},
           "kernels": kernels}
    with open(out, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    print(json.dumps({"written": out, "kernels": len(kernels), "fetch_scale": f_scale, "write_scale": w_scale}))


def _trace_rows(d):
    """(kernel name, dispatches, summed ns) from the rocpd database of a
    rocprofv3 --kernel-trace run (its `kernels` view)."""
    import sqlite3
    out = {}
    dbs = glob.glob(os.path.join(d, "**", "*.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no rocpd database (*.db) under {d}")
    for fn in dbs:
        con = sqlite3.connect(fn)
        for name, cnt, ns in con.execute("select name, count(*), sum(end - start) from kernels group by name"):
            k = _short(name)
            c0, n0 = out.get(k, (0, 0))
            out[k] = (c0 + cnt, n0 + ns)
        con.close()
    return out


def call_rate(trace, traffic, steps):
    """%HBM of whole coloring calls, every dispatch counted: each kernel's
    counter bytes per launch times its dispatches in one step of the counter
    run, over one step's summed kernel time in a kernel trace of the same
    workload (`trace`: name -> (dispatches, ns) over `steps` steps).  The
    runtime's own copy and fill kernels and torch's kernels (the counter
    calibration) are left out of both sums; a kernel the trace lacks makes
    the result None."""
    total_b = total_ns = 0
    kernels = []
    for k, v in traffic["kernels"].items():
        if k.startswith("__amd_rocclr") or k.startswith("at::"):
            continue
        t = trace.get(k)
        if t is None:
            # long template names are cut at different places by the two tools
            t = next((tv for tk, tv in trace.items() if tk[:60] == k[:60]), None)
        if t is None:
            return None
        total_b += int(v["hbm_bytes_per_launch"]) * int(v["dispatches"])
        total_ns += t[1] / steps
        kernels.append(k)
    if total_ns == 0:
        return None
    gbs = total_b / total_ns
    return {"bytes_per_step": int(total_b), "kernel_ms_per_step": round(total_ns / 1e6, 3),
            "gb_per_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "kernels": len(kernels)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-d2pd2", action="store_true", help="d1: skip the D2 + PD2 block of the line")
    ap.add_argument("--no-extras", action="store_true",
                    help="d1: skip the recolorDegrees and copy-ceiling blocks (after the timed steps), so that a "
                         "profile of the run holds the timed steps' kernels only")
    ap.add_argument("--workload", default="d1", choices=["d1", "d2pd2", "batch", "serve", "ghost", "dist", "ghost2"])
    ap.add_argument("--ghost-scale", type=int, default=24, help="ghost: R-MAT scale of the partitioned graph")
    ap.add_argument("--jobs", type=int, default=300, help="batch/serve: jobs in the stream")
    ap.add_argument("--n-max", type=float, default=3e4, help="batch/serve: largest job size (vertices)")
    ap.add_argument("--stream-seed", type=int, default=5)
    ap.add_argument("--slots", type=int, default=256, help="serve: job slots")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (for counter scaling)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--pmc-out", default=None, help="default: the workload's profiles/pmc_traffic*.json")
    ap.add_argument("--call-rate", nargs=2, metavar=("TRACE_DIR", "STEPS"),
                    help="%%HBM of whole calls from a kernel-trace run of STEPS steps (warm-up included) "
                         "and the workload's committed counter summary")
    args = ap.parse_args()
    if args.call_rate:
        with open(traffic_file(args.workload)) as f:
            traffic = json.load(f)
        r = call_rate(_trace_rows(args.call_rate[0]), traffic, int(args.call_rate[1]))
        print(json.dumps({"workload": args.workload, "source_hash": traffic.get("source_hash"), "call_rate": r}))
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload,
                      args.pmc_out or traffic_file(args.workload))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2107_00075_amd as gc

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.workload == "batch":
        out = bench_batch(args, torch, gc, dev)
    elif args.workload == "serve":
        out = bench_serve(args, torch, gc, dev)
    elif args.workload == "ghost":
        out = bench_ghost(args, torch, gc, dev)
    elif args.workload == "dist":
        out = bench_dist(args, torch, gc, dev)
    elif args.workload == "ghost2":
        out = bench_ghost2(args, torch, gc, dev)
    elif args.workload == "d2pd2":
        out = bench_d2pd2(args, torch, gc, dev)
    else:
        out = bench_d1(args, torch, gc, dev)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
