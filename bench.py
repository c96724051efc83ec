"""Benchmark of the dense-matrix Dijkstra hot path on one MI355X.

One step = one single-source solve (the whole n-iteration loop of Algorithm 1:
argmin, settle, relax row u into dist/pred, writeback) of the n=65536
undirected G(n, 0.5) graph with weights in [1, 1000] (16 GiB int32 matrix,
resident in HBM before timing), source 0.  `value` = matrix entries scanned
per second = n * (rows relaxed) / time per step.

The same JSON line carries the other workloads: n=16384 (undirected and
directed, sources 0/7/12345), n=1024 latency, and the batched launch of 320
instances against one-solve-per-launch; plus the HBM roofline of the
whole-GPU kernel and the CPU oracle timed on a bounded sample.
"""
import argparse
import gc
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INF_I32 = 0x7FFFFFFF
HBM_PEAK_GBS = 8000.0


SECTIONS = ("medium", "many_levels", "sparse", "small", "batched", "served")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--only-large", action="store_true", help="time only the n=65536 workload")
    ap.add_argument("--cpu-iters", type=int, default=32768,
                    help="iterations of the oracle timed for the CPU baseline")
    ap.add_argument("--serve-queries", type=int, default=20000,
                    help="queries of the served trace (Poisson arrivals at 2000/s)")
    ap.add_argument("--plain-queries", type=int, default=2000,
                    help="queries of the trace replayed one solve per launch for comparison")
    ap.add_argument("--section", choices=SECTIONS,
                    help="run only this part of the benchmark and print its figures (no headline line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 4 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def timed_solves(sp, torch, Wt, src, steps, warmup, flags=0, balance=0):
    n = Wt.shape[0]
    dist = torch.empty(n, dtype=torch.int32, device=Wt.device)
    pred = torch.empty(n, dtype=torch.int32, device=Wt.device)
    for _ in range(warmup):
        sp.sssp_dense_solve_ex(Wt, Wt.stride(0), n, src, dist, pred, flags, balance=balance)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        sp.sssp_dense_solve_ex(Wt, Wt.stride(0), n, src, dist, pred, flags, balance=balance)
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    status, stats = sp.sssp_last_status()
    if status & 3:
        raise RuntimeError("kernel status %d" % status)
    return {"ms_per_step": wall / steps * 1e3, "kernel_ms": kern, "stats": stats,
            "dist": dist, "pred": pred}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def read_traffic(name):
    """HBM traffic per launch from a committed rocprofv3 counter summary, if its
    kernel-source hash matches the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t:
        return None
    from paper_2504_03667_amd.build import source_hash
    if m.group(1) != source_hash():
        return None
    return float(t.group(1))


def read_ceiling_GBps(sp, torch, buf, reps=10):
    """Read bandwidth a plain streaming kernel (sssp_stream_read: chunks claimed
    dynamically, so no XCD waits for another) reaches over the same device buffer:
    the practical ceiling of a solve that streams it once.  Mean over `reps`
    launches, timed with events on the stream they run on."""
    sp.sssp_stream_read(buf)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        sp.sssp_stream_read(buf)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    return buf.numel() * buf.element_size() / (ms * 1e-3) / 1e9


def median_launch_ms(torch, fn, reps=11):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2] * 1e3


def bench_medium(sp, torch, gen):
    """n=16384, p=0.01 (1 GiB), undirected and directed, sources 0/7/12345: the whole-GPU solve
    (and the label-correcting method beside it)."""
    wl2 = gen.workload_single_medium()
    med = []
    for gi, g in enumerate(wl2.graphs):
        Wm = gen.dense_device(g)
        for g2, src in wl2.instances:
            if g2 != gi:
                continue
            rr = timed_solves(sp, torch, Wm, src, 10, 2)
            kms = percentile(rr["kernel_ms"], 50)
            gbps = (4.0 * g.n * rr["stats"][1] + 8.0 * g.n) / (kms * 1e-3) / 1e9
            lc = timed_solves(sp, torch, Wm, src, 10, 2, flags=sp.SSSP_FLAG_LABEL_CORRECTING)
            med.append({"directed": g.directed, "src": src, "ms_per_solve": round(rr["ms_per_step"], 4),
                        "kernel_ms_median": round(kms, 4), "rows_relaxed": rr["stats"][1],
                        "rounds": rr["stats"][0],
                        "entries_per_s": g.n * rr["stats"][1] / (rr["ms_per_step"] * 1e-3),
                        "algorithmic_GBps": round(gbps, 1), "frac_hbm_peak": round(gbps / HBM_PEAK_GBS, 4),
                        "label_correcting": {"ms_per_solve": round(lc["ms_per_step"], 4),
                                             "sweeps": lc["stats"][0], "rows_streamed": lc["stats"][1]}})
            del lc
        del Wm
    return med


def bench_small(sp, torch, gen):
    """n=1024, p=0.1: latency of one solve, one workgroup and whole GPU."""
    g1 = gen.workload_single_small().graphs[0]
    W1 = gen.dense_device(g1)
    c1 = {}
    for mode, flags, reps in (("single_workgroup", 0, 1000), ("whole_gpu", sp.SSSP_FLAG_GRID, 200)):
        rr = timed_solves(sp, torch, W1, 0, reps, 10, flags=flags)
        med_us = 1e3 * percentile(rr["kernel_ms"], 50)
        c1[mode] = {"reps": reps, "median_us": round(med_us, 2),
                    "p99_us": round(1e3 * percentile(rr["kernel_ms"], 99), 2),
                    "rounds": rr["stats"][0], "rows_relaxed": rr["stats"][1],
                    "entries_per_s": g1.n * rr["stats"][1] / (med_us * 1e-6)}
    del W1
    return c1


def bench_many_levels(sp, torch, gen):
    """Graphs whose shortest paths take hundreds of distinct distances (sparse, weights
    in [1, 1000], like the sparse end of the served set): the Dijkstra rounds pay one
    barrier per distance, the label-correcting sweeps one per sweep."""
    out = []
    for n, p, seed in ((4096, 0.002, 11), (8192, 0.001, 12), (16384, 0.0005, 13), (32768, 0.0005, 14)):
        g = gen.GraphSpec(n, p, 1, 1000, gen.SEED_BASE + 100 + seed)
        W = gen.dense_device(g)
        row = {"n": n, "p": p, "weights": [1, 1000]}
        for name, flags in (("dijkstra", 0), ("dijkstra_one_workgroup", sp.SSSP_FLAG_SINGLE),
                            ("label_correcting", sp.SSSP_FLAG_LABEL_CORRECTING)):
            if flags == sp.SSSP_FLAG_SINGLE and n > sp.sssp_single_max_n():
                continue
            r = timed_solves(sp, torch, W, 0, 5, 1, flags=flags)
            row[name] = {"ms_per_solve": round(r["ms_per_step"], 3), "rounds": r["stats"][0],
                         "rows_streamed": r["stats"][1]}
        out.append(row)
        del W
    return out


def bench_sparse(sp, torch, gen):
    """The paper's sparse family (m = 3n undirected edges, weights in [1, 1000], source 0)
    as adjacency lists: device conversion of the edge list, the CSR solve, and for
    n <= 40000 the same graph as an n x n matrix (Dijkstra rounds and label-correcting)."""
    out = []
    _, specs = gen.workload_sparse()
    for s in specs:
        eu, ev, ew = (torch.from_numpy(a).cuda() for a in gen.sparse_edges(s.n, s.m, s.lo, s.hi, s.seed))
        conv_ms = median_launch_ms(torch, lambda: sp.csr_from_edges(eu, ev, ew, s.n, s.directed), reps=3)
        rp, col, w, _ = sp.csr_from_edges(eu, ev, ew, s.n, s.directed)
        ms = median_launch_ms(torch, lambda: sp.csr_solve(rp, col, w, 0))
        _, stats = sp.sssp_last_status()
        # device time of one solve (scratch allocation, init and solve kernels) from events on its stream
        dev_ms = []
        for _ in range(7):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            sp.csr_solve(rp, col, w, 0)
            e1.record()
            e1.synchronize()
            dev_ms.append(e0.elapsed_time(e1))
        dms = percentile(dev_ms, 50)
        row = {"n": s.n, "m": s.m, "lists_entries": int(col.numel()), "convert_ms": round(conv_ms, 3),
               "csr": {"ms_per_solve": round(ms, 3), "device_ms_median": round(dms, 3), "sweeps": stats[0],
                       "edge_lists_relaxed": stats[1], "us_per_sweep": round(1e3 * dms / max(1, stats[0]), 2),
                       "edges_per_s": col.numel() / (ms * 1e-3)}}
        if s.n <= 40000:
            W = torch.empty((s.n, s.n), dtype=torch.int32, device="cuda")
            sp.sssp_edges_to_dense(eu, ev, ew, s.n, W, directed=s.directed)
            for name, flags in (("dense_dijkstra", 0), ("dense_label_correcting", sp.SSSP_FLAG_LABEL_CORRECTING)):
                r = timed_solves(sp, torch, W, 0, 3, 1, flags=flags)
                row[name] = {"ms_per_solve": round(r["ms_per_step"], 3), "rounds": r["stats"][0],
                             "rows_streamed": r["stats"][1]}
            del W
        out.append(row)
        del eu, ev, ew, rp, col, w
        torch.cuda.empty_cache()
    return out


def bench_batched(sp, torch, gen):
    """256 sources on one n=8192 graph plus 64 graphs: one-shot launch, autotuned plans
    (int32 and exact compact copies, replayed as a hipGraph) and one solve per launch."""
    wl = gen.workload_batched()
    mats = [gen.dense_device(g) for g in wl.graphs]
    items = []
    for gi, src in wl.instances:
        nn = wl.graphs[gi].n
        items.append((mats[gi], src, torch.empty(nn, dtype=torch.int32, device="cuda"),
                      torch.empty(nn, dtype=torch.int32, device="cuda")))
    res = {"instances": len(items)}
    t_one = median_launch_ms(torch, lambda: sp.sssp_dense_solve_batched(items))
    status, bstats = sp.sssp_last_status()
    res["one_shot"] = {"launch_ms": round(t_one, 3), "solves_per_s": round(len(items) / t_one * 1e3, 1),
                       "status": status}
    ref = [(d.cpu().numpy().copy(), p.cpu().numpy().copy()) for _, _, d, p in items]
    # algorithmic bytes of one launch: each instance streams its reachable vertices'
    # rows (n entries each) once; entries are 4 bytes, or 1 / 2 in exact compact copies
    reach = [int((a != INF_I32).sum()) for a, _ in ref]
    elem = []
    for W_ in mats:
        _, mx = sp.sssp_dense_validate(W_, W_.stride(0), W_.shape[0])
        elem.append(1 if mx <= 254 else 2 if mx <= 65534 else 4)
    inst_graph = [gi for gi, _ in wl.instances]
    alg = {0: sum(4.0 * wl.graphs[g].n * r for g, r in zip(inst_graph, reach)),
           sp.SSSP_FLAG_COMPACT: sum(float(elem[g]) * wl.graphs[g].n * r for g, r in zip(inst_graph, reach))}
    res["one_shot"]["algorithmic_GBps"] = round(alg[0] / (t_one * 1e-3) / 1e9, 1)
    for name, flags in (("plan_int32", 0), ("plan_compact", sp.SSSP_FLAG_COMPACT)):
        with sp.BatchPlan(items, flags) as plan:
            t = median_launch_ms(torch, plan.launch)
            st, _ = plan.status()
            info = plan.info()
            same = all(np.array_equal(d.cpu().numpy(), a) and np.array_equal(p.cpu().numpy(), b)
                       for (_, _, d, p), (a, b) in zip(items, ref))
        res[name] = {"launch_ms": round(t, 3), "solves_per_s": round(len(items) / t * 1e3, 1), "status": st,
                     "identical_to_one_shot": same, "single_max_n": info["single_max_n"],
                     "gang_columns": info["gang_columns"], "candidates": info["candidates"],
                     "compact_graphs": info["compact_graphs"], "build_ms": round(info["build_ms"], 1),
                     "group_sources": info["group_sources"], "group_columns": info["group_columns"],
                     "group_items": info["group_items"],
                     "algorithmic_GBps": round(alg[flags] / (t * 1e-3) / 1e9, 1)}
    # plain path: one sssp_dense_solve per instance, synchronised each time
    t0 = time.perf_counter()
    for W_, src, dist_, pred_ in items:
        sp.sssp_dense_solve_ex(W_, W_.stride(0), W_.shape[0], src, dist_, pred_, 0)
        torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    plain = len(items) / tp
    res["plain_solves_per_s"] = round(plain, 1)
    res["rows_relaxed"] = bstats[1]
    for name in ("one_shot", "plan_int32", "plan_compact"):
        res[name]["speedup_vs_plain"] = round(res[name]["solves_per_s"] / plain, 2)
    # a plan pays for its build (compact copies, autotuning, capture) over its launches:
    # the speedup with the build spread over 100 launches, and the launches it takes
    # until the plan (build included) has beaten solving one instance per launch
    plain_batch_ms = len(items) / plain * 1e3
    for name in ("plan_int32", "plan_compact"):
        r = res[name]
        r["speedup_vs_plain_build_over_100_launches"] = round(
            plain_batch_ms * 100 / (r["build_ms"] + 100 * r["launch_ms"]), 2)
        gain = plain_batch_ms - r["launch_ms"]
        r["launches_to_repay_build"] = round(r["build_ms"] / gain, 2) if gain > 0 else None
    del mats, items
    return res


def bench_served(sp, torch, gen, args):
    """Replays the served workload: open-loop Poisson arrivals (latency = host-observed
    completion minus the scheduled arrival), then all queries released at once
    (saturation throughput), then a prefix of the trace one solve per launch."""
    wl = gen.workload_serving(n_queries=args.serve_queries)
    mats = [gen.dense_device(g) for g in wl.graphs]
    outs = [(torch.empty(wl.graphs[q.graph].n, dtype=torch.int32, device="cuda"),
             torch.empty(wl.graphs[q.graph].n, dtype=torch.int32, device="cuda")) for q in wl.queries]
    torch.cuda.synchronize()
    res = {"graphs": len(wl.graphs), "queries": len(wl.queries), "offered_qps": 2000.0}
    for name, flags, replay in (("server_int32", 0, False), ("server_compact", sp.SSSP_FLAG_COMPACT, True)):
        print("[bench] served %s: %d queries" % (name, len(wl.queries)), file=sys.stderr, flush=True)
        r = {}
        with sp.Server() as srv:
            gids = [srv.add_graph(W, flags) for W in mats]
            r["graphs_compact"] = sum(1 for g in gids if srv.graph_elem(g) < 4)
            warm = [srv.submit(gids[q.graph], q.src, d, p) for q, (d, p) in list(zip(wl.queries, outs))[:64]]
            for t in warm:
                srv.wait(t, timeout_s=120)
            srv.poll(1 << 20)
            if replay:
                # open-loop replay: latency = host-observed completion - scheduled arrival
                # (Python's garbage collector is paused meanwhile: its pauses would
                # delay submissions, a property of this harness, not of the server)
                gc.collect()
                gc.disable()
                t0 = sp.sssp_server_now_ns() + 2_000_000
                tickets = []
                for q, (d, p) in zip(wl.queries, outs):
                    target = t0 + int(q.arrival_s * 1e9)
                    while sp.sssp_server_now_ns() < target:
                        pass
                    tickets.append(srv.submit(gids[q.graph], q.src, d, p))
                for t in tickets:
                    srv.wait(t, timeout_s=300)
                gc.enable()
                lat, svc, t_end, bad = [], [], 0, 0
                for q, t in zip(wl.queries, tickets):
                    inf = srv.info(t)
                    bad += inf["status"] & 3
                    lat.append((inf["t_done_ns"] - (t0 + int(q.arrival_s * 1e9))) / 1e3)
                    svc.append((inf["t_done_ns"] - inf["t_admit_ns"]) / 1e3)
                    t_end = max(t_end, inf["t_done_ns"])
                r["replay"] = {"p50_us": round(percentile(lat, 50), 1), "p99_us": round(percentile(lat, 99), 1),
                               "mean_us": round(sum(lat) / len(lat), 1), "max_us": round(max(lat), 1),
                               "admitted_to_done_p50_us": round(percentile(svc, 50), 1),
                               "admitted_to_done_p99_us": round(percentile(svc, 99), 1),
                               "solves_per_s": round(len(tickets) / ((t_end - t0) / 1e9), 1), "bad_status": bad}
                # one query per graph with the server otherwise idle: the latency floor
                alone = []
                for gi in range(len(wl.graphs)):
                    q = next((q for q in wl.queries if q.graph == gi), None)
                    if q is None:
                        continue
                    d, p = outs[wl.queries.index(q)]
                    t = srv.submit(gids[gi], q.src, d, p)
                    srv.wait(t, timeout_s=120)
                    inf = srv.info(t)
                    alone.append(((inf["t_done_ns"] - inf["t_submit_ns"]) / 1e3, gi, inf["rounds"], inf["parts"]))
                alone.sort()
                r["alone"] = {"graphs": len(alone), "median_us": round(alone[len(alone) // 2][0], 1),
                              "slowest": [{"us": round(a, 1), "n": wl.graphs[gi].n, "p": round(wl.graphs[gi].p, 5),
                                           "rounds": rd, "parts": pt} for a, gi, rd, pt in alone[-4:]]}
            # saturation: every query released at once
            ts = sp.sssp_server_now_ns()
            tickets = [srv.submit(gids[q.graph], q.src, d, p) for q, (d, p) in zip(wl.queries, outs)]
            for t in tickets:
                srv.wait(t, timeout_s=300)
            infos = [srv.info(t) for t in tickets]
            te = max(i["t_done_ns"] for i in infos)
            elem = [srv.graph_elem(g) for g in gids]  # bytes per stored entry (compact copies: 1 or 2)
            rows = sum(i["settled"] * wl.graphs[q.graph].n * elem[q.graph] for q, i in zip(wl.queries, infos))
            r["saturation"] = {"solves_per_s": round(len(tickets) / ((te - ts) / 1e9), 1),
                               "seconds": round((te - ts) / 1e9, 3),
                               "bad_status": sum(i["status"] & 3 for i in infos),
                               "algorithmic_GBps": round(rows / ((te - ts) / 1e9) / 1e9, 1)}
            r["workgroups"] = srv.stats()["workgroups"]
        res[name] = r
    # one solve per launch, synchronised each time, over a prefix of the trace
    k = min(args.plain_queries, len(wl.queries))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, (d, p) in list(zip(wl.queries, outs))[:k]:
        W = mats[q.graph]
        sp.sssp_dense_solve_ex(W, W.stride(0), W.shape[0], q.src, d, p, 0)
        torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    res["plain"] = {"queries": k, "solves_per_s": round(k / tp, 1)}
    # the same prefix replayed at its scheduled arrivals, one solve per launch: the plain
    # path cannot keep up with 2000 queries/s, so its latency grows along the trace
    lat = []
    t0 = time.perf_counter() + 0.002
    for q, (d, p) in list(zip(wl.queries, outs))[:k]:
        arrive = t0 + q.arrival_s
        while time.perf_counter() < arrive:
            pass
        W = mats[q.graph]
        sp.sssp_dense_solve_ex(W, W.stride(0), W.shape[0], q.src, d, p, 0)
        torch.cuda.current_stream().synchronize()
        lat.append((time.perf_counter() - arrive) * 1e6)
    res["plain"]["replay"] = {"queries": k, "p50_us": round(percentile(lat, 50), 1),
                              "p99_us": round(percentile(lat, 99), 1), "max_us": round(max(lat), 1)}
    # literal mode of the plain path (one vertex per step, as Algorithm 1 is printed)
    kl = min(30, len(wl.queries))
    t0 = time.perf_counter()
    for q, (d, p) in list(zip(wl.queries, outs))[:kl]:
        W = mats[q.graph]
        sp.sssp_dense_solve_ex(W, W.stride(0), W.shape[0], q.src, d, p, sp.SSSP_FLAG_LITERAL)
        torch.cuda.current_stream().synchronize()
    tl = time.perf_counter() - t0
    res["plain_literal"] = {"queries": kl, "solves_per_s": round(kl / tl, 2)}
    for name in ("server_int32", "server_compact"):
        res[name]["saturation_speedup_vs_plain"] = round(res[name]["saturation"]["solves_per_s"] / (k / tp), 2)
        res[name]["saturation_speedup_vs_plain_literal"] = round(
            res[name]["saturation"]["solves_per_s"] / (kl / tl), 1)
    del mats, outs
    return res


def host_cpu():
    """The host CPU as the process sees it: lscpu's model and topology, the cores the
    process may run on (its affinity) and its cgroup CPU quota; usable_cores is the
    smaller of the two, the threads the CPU baselines use."""
    info = {"nproc": len(os.sched_getaffinity(0)), "model": "", "lscpu": {}}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            k, v = k.strip(), v.strip()
            if k in ("Model name", "Vendor ID", "CPU family", "Model", "Socket(s)", "Core(s) per socket",
                     "Thread(s) per core", "CPU(s)", "CPU max MHz", "L3"):
                info["lscpu"][k] = v
        info["model"] = info["lscpu"].get("Model name", "")
    except (OSError, subprocess.SubprocessError):
        pass
    quota = None
    try:
        q, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = int(q) / int(period)
    except (OSError, ValueError):
        pass
    info["cgroup_cpu_quota"] = quota
    info["usable_cores"] = max(1, min(info["nproc"], int(quota) if quota else info["nproc"]))
    return info


def cpu_throughput(gen):
    """Independent oracle solves spread over every host core (one solve per thread), on
    samples of the batched and served instance sets: CPU solves/s for context."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    host = host_cpu()
    cores = host["usable_cores"]
    out = {"cores": cores, "cpu_model": host["model"], "host": host, "kind": "oracle"}
    for name, wl, per_core in (("batched", gen.workload_batched(), 32), ("served", gen.workload_serving(n_queries=400), 12)):
        pairs = wl.instances if wl.instances else [(q.graph, q.src) for q in wl.queries]
        rng = np.random.default_rng(7)
        pick = [pairs[i] for i in rng.permutation(len(pairs))[:per_core * cores]]
        need = sorted({g for g, _ in pick})
        host = {g: gen.dense_host(wl.graphs[g]) for g in need}
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda gs: oracle.dijkstra(host[gs[0]], gs[1]), pick))
        dt = time.perf_counter() - t0
        out[name] = {"solves_per_s": round(len(pick) / dt, 2), "sample": "%d instances drawn from the set" % len(pick),
                     "seconds": round(dt, 2)}
        del host
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the dense-matrix Dijkstra path runs on a single "
              "MI355X (--gpus %d requested); column sharding across GPUs is not implemented." % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import gen
    import paper_2504_03667_amd as sp

    sp.lib()
    if args.copy_calibration:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        a = torch.empty(1 << 30, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.section:
        run = {"medium": bench_medium, "many_levels": bench_many_levels, "sparse": bench_sparse,
               "small": bench_small, "batched": bench_batched,
               "served": lambda sp, torch, gen: bench_served(sp, torch, gen, args)}[args.section]
        print(json.dumps({"section": args.section, args.section: run(sp, torch, gen)}))
        return 0

    # ---- n = 65536, p = 0.5, 16 GiB: the headline -------------------------------
    wl = gen.workload_single_large()
    spec = wl.graphs[0]
    print("[bench] generating n=%d matrix on the GPU" % spec.n, file=sys.stderr, flush=True)
    Wt = gen.dense_device(spec)
    torch.cuda.synchronize()
    print("[bench] timing %d steps (+%d warmup)" % (args.steps, args.warmup), file=sys.stderr, flush=True)
    r = timed_solves(sp, torch, Wt, 0, args.steps, args.warmup)
    trace = sp.sssp_last_trace()
    n = spec.n
    R = r["stats"][1]
    rounds = r["stats"][0]
    entries = n * R
    ms = r["ms_per_step"]
    kern_ms = sum(r["kernel_ms"]) / len(r["kernel_ms"])
    alg_bytes = 4.0 * n * R + 8.0 * n
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = read_traffic("k_grid_n65536_counters.txt")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_grid (whole-GPU persistent solve)", "kernel_ms": round(kern_ms, 4),
                "algorithmic_bytes_per_launch": alg_bytes}
    # the same 16 GiB read by a kernel that does nothing else: what the chip delivers
    ceiling = read_ceiling_GBps(sp, torch, Wt)
    roofline["read_ceiling_GBps"] = round(ceiling, 1)
    roofline["frac_of_read_ceiling"] = round(achieved / ceiling, 4)
    round_us = [round((trace[i + 1][0] - trace[i][0]) / 1e3, 1) for i in range(len(trace) - 1)]
    large = {"n": n, "rows_relaxed": R, "rounds": rounds, "barriers": r["stats"][3],
             "round_rows": [t[1] for t in trace[:-1]], "round_us": round_us,
             "ms_per_solve": round(ms, 4), "entries_per_s": entries / (ms * 1e-3),
             "algorithmic_GBps": round(alg_bytes / (ms * 1e-3) / 1e9, 1)}
    # the same solves without pair balancing of the large rounds (identical dist/pred)
    unb = timed_solves(sp, torch, Wt, 0, max(3, args.steps // 2), 1, balance=-1)
    if not torch.equal(unb["dist"], r["dist"]) or not torch.equal(unb["pred"], r["pred"]):
        raise RuntimeError("dist/pred differ without pair balancing")
    large["kernel_ms_without_pair_balance"] = round(sum(unb["kernel_ms"]) / len(unb["kernel_ms"]), 4)
    del unb
    # literal mode once: one vertex per grid barrier (Algorithm 1 as printed)
    if not args.only_large:
        lit = timed_solves(sp, torch, Wt, 0, 1, 0, flags=sp.SSSP_FLAG_LITERAL)
        large["literal_ms_per_solve"] = round(lit["ms_per_step"], 2)
        large["literal_us_per_barrier"] = round(lit["ms_per_step"] * 1e3 / max(1, lit["stats"][3]), 3)
        del lit
    dist_large = r["dist"].cpu().numpy()
    del Wt, r
    torch.cuda.empty_cache()

    extra = {}
    if not args.only_large:
        extra["n16384"] = bench_medium(sp, torch, gen)
        torch.cuda.empty_cache()

        # ---- sparse graphs with wide weights: Dijkstra rounds vs label-correcting ----
        extra["many_levels"] = bench_many_levels(sp, torch, gen)
        torch.cuda.empty_cache()

        # ---- the sparse family (m = 3n) as adjacency lists ------------------------
        print("[bench] sparse graphs as adjacency lists", file=sys.stderr, flush=True)
        extra["sparse_m3n"] = bench_sparse(sp, torch, gen)

        extra["n1024"] = bench_small(sp, torch, gen)

        # ---- batched: 320 instances in one launch vs one solve per launch ---------
        extra["batched"] = bench_batched(sp, torch, gen)
        torch.cuda.empty_cache()

        # ---- served: 32 resident graphs, Poisson trace, continuous batching --------
        extra["served"] = bench_served(sp, torch, gen, args)
        torch.cuda.empty_cache()

        # ---- CPU oracle over all host cores on samples of the batched / served sets --
        if not args.skip_cpu:
            extra["cpu_batched_served"] = cpu_throughput(gen)

    # ---- CPU oracle on a bounded sample of the headline workload -----------------
    cpu = None
    if not args.skip_cpu:
        import oracle
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        Wh = gen.dense_host(spec)
        t0 = time.perf_counter()
        rel = oracle.dijkstra_prefix(Wh, 0, args.cpu_iters)
        dt = time.perf_counter() - t0
        host = host_cpu()
        cpu = {"value": n * rel / dt, "unit": "matrix entries scanned/s", "cores": 1, "kind": "oracle",
               "sample": "first %d of %d iterations of Algorithm 1 (serial C, one thread) on the "
                         "n=65536 p=0.5 source-0 solve, %.1f s" % (args.cpu_iters, n, dt),
               "cpu_model": host["model"], "nproc": host["nproc"], "cgroup_cpu_quota": host["cgroup_cpu_quota"]}
        del Wh

    line = {
        "metric": "matrix entries scanned/s (single-source dense Dijkstra, n=65536)",
        "value": entries / (ms * 1e-3),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic: seeded counter-based G(n,p) matrices generated in HBM",
        "config": {"workload": wl.name, "n": n, "p": spec.p, "weights": [spec.lo, spec.hi],
                   "directed": spec.directed, "src": 0, "matrix_bytes": 4 * n * n,
                   "parallelism": "single GPU, persistent cooperative grid"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "large": large,
    }
    line.update(extra)
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
