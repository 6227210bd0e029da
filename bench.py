"""Benchmark: generic worst-case optimal join with aggregation on one MI355X.

Default workload: triangle COUNT  R(a,b) |x| S(b,c) |x| T(a,c)  on an R-MAT
graph with 2^22 vertices and 2^26 sampled edges (a=0.57, b=0.19, c=0.19),
edges oriented low->high and deduplicated by the set-mode trie build.

One step is one pass of the whole path over the resident edge list:
lh_trie_build (sort, dedup, levels, layouts) + lh_plan (order, policies)
+ lh_join_aggregate (multiway intersections, COUNT) + reading the count.
value = join-aggregate input tuples per second = 3 * |E'| / step time (the
three atoms each hold the |E'| deduplicated edges).

The same steps are timed twice on the same graph: under the plain rules of
section 4 (plain layout, plain order), then under the learned cost model
(learned layouts and order, committed weights); the learned run is the
reported value, the plain run and the ratio sit in the config.  Results of
both must be identical.

Prints one JSON line.
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "join-aggregate tuples/s + HBM GB/s, learned+batched vs plain WCOJ, 1 GPU"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def leaf_model_bytes(rows, elements):
    """The leaf's own byte model (a second figure next to the minimum): per
    frontier row its two trie positions (8 B), the two sets' child ranges
    (16 B), its work offset (8 B) and driver id (1 B); per element of the
    smaller set the element itself (4 B) and one probe of the other set
    (4 B)."""
    return 33 * rows + 8 * elements


def triangle_min_bytes(edges, wedges, n_vertices):
    """Bytes a worst-case optimal triangle COUNT cannot avoid moving under
    the order a, b, c: the set S(b) is streamed once for every edge (a, b)
    that reaches it (4 B per wedge, sum over edges of the out-degree of b),
    the set T(a) is read once per a (4 B per edge), and the level-0 child
    offsets once (8 B per vertex + 1).  The sum over edges (a, b) of d+(b)
    equals sum over b of d-(b) d+(b), so the reversed order c, b, a has the
    same minimum."""
    return 4 * wedges + 4 * edges + 8 * (n_vertices + 1)


# profiling scope -> the kernel it times (the two-set COUNT leaf of the triangle)
KERNEL_OF_SCOPE = {"leaf_aggregate": "k_leaf2_count"}
# HBM bytes per launch of that kernel from rocprofv3 counters, used only
# while the kernel's source matches the one the counters saw
TRAFFIC_SUMMARY = {"plain": "triangle_rmat22_plain_leaf_traffic.txt",
                   "learned": "triangle_rmat22_learned_leaf_traffic.txt"}
# the two-set leaf's launches: every row but those of the two buckets, the
# top bucket, the merged rows
LEAF_SCOPES = ("leaf_aggregate", "leaf_top", "leaf_merge")
FLUSH_BYTES = 512 << 20      # more than the 256 MB Infinity Cache and the 8 x 4 MB L2


def edge_stats(torch, lo_d, hi_d):
    """Deduplicated oriented edges E', wedges W = sum over edges (a, b) of
    d+(b), and the streamed elements sum over edges of d+(a) + d+(b), from
    the resident edge columns (torch on the device; measurement only)."""
    lo = lo_d.to(torch.int64) & 0xffffffff
    hi = hi_d.to(torch.int64) & 0xffffffff
    u = torch.unique((lo << 32) | hi)
    ul, uh = u >> 32, u & 0xffffffff
    n = int(torch.maximum(ul.max(), uh.max()).item()) + 1
    dout = torch.bincount(ul, minlength=n)
    din = torch.bincount(uh, minlength=n)
    wedges = int((dout * din).sum().item())
    stream = int((dout[ul] + dout[uh]).sum().item())
    e = int(u.numel())
    del lo, hi, u, ul, uh, dout, din
    return e, wedges, stream


def run_protocol(torch, step, flush=None, runs=7):
    """The paper's timing protocol (section 6.1): `runs` runs, the fastest
    and the slowest dropped, the mean of the rest; plus the median.  With
    `flush`, a 512 MB write evicts the caches before every run (cold)."""
    times = []
    for _ in range(runs):
        if flush is not None:
            flush.add_(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1000)
    s = sorted(times)
    mid = s[1:-1] if runs >= 3 else s
    return {"mean_drop_minmax_ms": round(sum(mid) / len(mid), 3), "median_ms": round(s[len(s) // 2], 3),
            "min_ms": round(s[0], 3), "max_ms": round(s[-1], 3), "runs": runs}


def cpu_baseline(scale, headline):
    """The oracle (pairwise hash join, OpenMP over its probe side) on the
    host cores, on an R-MAT graph of the same recipe at a smaller scale.
    The headline graph's wedge count is printed first: the pairwise join
    would materialize that many intermediate tuples."""
    import oracle
    import synth
    from tests import queries
    lo, hi = synth.rmat_edges(scale, 16 << scale, seed=2)
    key = np.unique(lo.astype(np.uint64) << np.uint64(32) | hi.astype(np.uint64))
    ulo = (key >> np.uint64(32)).astype(np.int64)
    uhi = (key & np.uint64(0xffffffff)).astype(np.int64)
    n = 1 << scale
    w = int((np.bincount(ulo, minlength=n) * np.bincount(uhi, minlength=n)).sum())
    e = len(key)
    del key, ulo, uhi
    log(f"cpu baseline: the headline graph has W = {headline['wedges']} wedges "
        f"({headline['wedges'] * 20 / 1e12:.2f} TB of pairwise intermediate at 20 B per tuple); "
        f"the oracle runs R-MAT {scale}: E' = {e}, W = {w}")
    q = queries.triangle(lo, hi)
    threads = oracle.threads()
    t0 = time.perf_counter()
    res = oracle.join_aggregate(q)
    dt = time.perf_counter() - t0
    log(f"  oracle: {dt:.1f} s on {threads} threads, {int(res['counts'][0])} triangles")
    return {"value": 3 * e / dt, "unit": "tuples/s", "cores": threads, "kind": "oracle",
            "sample": f"R-MAT scale {scale} (2^{scale} vertices, {16 << scale} samples, same a,b,c, seed 2): "
                      f"E' = {e} edges, W = {w} wedges materialized by the pairwise join, full triangle COUNT = "
                      f"{int(res['counts'][0])}, one run of {dt:.1f} s on {threads} OpenMP threads; the headline "
                      f"graph (W = {headline['wedges']}) is beyond the oracle's memory",
            "wedges": w, "edges": e, "seconds": round(dt, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--samples-log2", type=int, default=26)
    ap.add_argument("--cpu-scale", type=int, default=18)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--runs", type=int, default=7,
                    help="runs of the timing protocol (min and max dropped); 0 skips it")
    ap.add_argument("--batch-policies", default="plain,learned",
                    help="policies of the batch legs (comma-separated)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batch: time the batched launch only (e.g. to profile the graph launch alone)")
    ap.add_argument("--no-side", action="store_true",
                    help="time the headline triangle only (no SpGEMM, no batch legs)")
    ap.add_argument("--layout", default="plain", choices=["plain", "uint", "bitset", "learned"],
                    help="layout of the plain-policy run")
    ap.add_argument("--policy", default="both", choices=["both", "plain", "learned"],
                    help="both: time the plain rule, then the learned cost model (reported)")
    ap.add_argument("--workload", default="triangle", choices=["triangle", "batch", "learned", "copy", "gather", "intersect", "q5", "groupby", "dense",
                             "spgemm-star", "voter", "configs"])
    ap.add_argument("--weights", default=None)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--card", type=int, default=1_000_000)
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--sf", type=float, default=10.0)
    ap.add_argument("--voters", type=int, default=7_503_555)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU layout is a design "
              "note only", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1708_07859_amd import lh

    torch.cuda.set_device(0)
    # Python's cyclic collector would otherwise traverse every object torch
    # and numpy created at import, tens of milliseconds per full pass, at
    # a moment set by allocation counts (which differ when imports compile
    # their sources): the objects alive now are frozen out of collection,
    # and timed loops run with the collector paused, as timeit does.
    gc.collect()
    gc.freeze()
    if args.workload == "batch":
        return bench_batch(args, lh, torch, synth)
    if args.workload == "learned":
        return bench_learned(args, lh, torch, synth)
    if args.workload == "copy":
        return bench_copy(args, torch)
    if args.workload == "gather":
        return bench_gather(args, torch)
    if args.workload == "configs":
        return bench_configs(args, lh, torch, synth)
    if args.workload == "intersect":
        return bench_intersect(args, lh, torch, synth)
    if args.workload == "q5":
        return bench_q5(args, lh, torch, synth)
    if args.workload == "groupby":
        return bench_groupby(args, lh, torch, synth)
    if args.workload == "dense":
        return bench_dense(args, lh, torch, synth)
    if args.workload == "spgemm-star":
        return bench_spgemm_star(args, lh, torch, synth)
    if args.workload == "voter":
        return bench_voter(args, lh, torch, synth)
    log(f"generating R-MAT scale {args.scale}, 2^{args.samples_log2} samples")
    t0 = time.perf_counter()
    lo, hi = synth.rmat_edges(args.scale, 1 << args.samples_log2, seed=2)
    log(f"  {len(lo)} oriented samples in {time.perf_counter() - t0:.1f} s")
    lo_d = lh.to_device(lo)
    hi_d = lh.to_device(hi)
    del lo, hi
    torch.cuda.synchronize()
    n_edges, wedges, streamed = edge_stats(torch, lo_d, hi_d)
    b_min = triangle_min_bytes(n_edges, wedges, 1 << args.scale)
    log(f"  E' = {n_edges} edges, W = {wedges} wedges, streamed elements {streamed}, minimum bytes {b_min}")
    flush = torch.empty(FLUSH_BYTES, dtype=torch.uint8, device="cuda").zero_()

    runs = {}
    policies = ["plain", "learned"] if args.policy == "both" else [args.policy]
    for policy in policies:
        layout = args.layout if policy == "plain" else "learned"
        if policy == "learned":
            from paper_1708_07859_amd import learned as L
            lm, om, _ = L.load(args.weights or L.DEFAULT_WEIGHTS)
            L.register(lm, om)
        runs[policy] = measure_triangle(args, lh, torch, lo_d, hi_d, layout, policy, flush)
        if policy == "learned":
            lh.use_model(lh.LH_MODEL_LAYOUT, None)
            lh.use_model(lh.LH_MODEL_ORDER, None)
    head_policy = policies[-1]
    head = runs[head_policy]
    if len(runs) == 2:
        assert runs["plain"]["count"] == runs["learned"]["count"], "policies disagree on the count"
    prof = head["prof"]
    # roofline of the dominant kernel, the two-set leaf: its main launch plus
    # the top-bucket launch, per step
    roof = None
    if "leaf_aggregate" in prof:
        e = prof["leaf_aggregate"]
        top = prof.get("leaf_top", {"total_ms": 0.0, "launches": 0})
        avg_ms = sum(prof[k]["total_ms"] for k in LEAF_SCOPES if k in prof) / e["launches"]
        achieved = b_min / (avg_ms / 1000) / 1e9
        model_bytes = leaf_model_bytes(e["rows"], e["elements"]) / e["launches"]
        kernel = KERNEL_OF_SCOPE["leaf_aggregate"]
        traffic = None
        top_traffic = None
        summary = TRAFFIC_SUMMARY.get(head_policy)
        if summary and (args.scale, args.samples_log2) == (22, 26) and (head_policy != "plain" or args.layout == "plain"):
            from paper_1708_07859_amd import profiling
            path = os.path.join(ROOT, "profiles", summary)
            # every launch of the leaf that ran needs its counters
            parts = [profiling.read_traffic(path, kernel)]
            for scope, name in (("leaf_top", kernel + "_top"), ("leaf_merge", "k_leaf2_merge")):
                if scope in prof:
                    parts.append(profiling.read_traffic(path, name))
                    if scope == "leaf_top":
                        top_traffic = parts[-1]
            traffic = None if any(x is None for x in parts) else sum(parts)
        top_ms = top["total_ms"] / e["launches"]
        # the top bucket (rows whose two sets hold 2^14 elements or more):
        # its own launch, timed with HIP events, its DRAM bytes from the
        # counters (L2 misses, reads in 32-byte requests + writes)
        top_bucket = None
        if top["launches"]:
            top_bucket = {"kernel": kernel + "<top>", "ms_per_launch": round(top_ms, 4),
                          "units_per_launch": top.get("rows", 0) // max(1, top["launches"]),
                          "dram_bytes": None if top_traffic is None else int(top_traffic),
                          "dram_GBs": None if top_traffic is None else round(top_traffic / (top_ms / 1000) / 1e9, 1),
                          "dram_frac": None if top_traffic is None else
                          round(top_traffic / (top_ms / 1000) / 1e9 / HBM_PEAK_GBS, 4)}
        roof = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "avg_launch_ms": round(avg_ms, 4), "top_bucket_ms": round(top_ms, 4), "top_bucket": top_bucket,
                "merge_ms": round(prof.get("leaf_merge", {"total_ms": 0.0})["total_ms"] / e["launches"], 4),
                "alg_bytes_per_launch": int(b_min),
                "alg_bytes": "minimum bytes: 4 B per wedge (S(b) streamed per edge) + 4 B per edge (T(a) once) + "
                             "8 B per vertex (offsets)",
                "model_bytes_per_launch": int(model_bytes),
                "model_frac": round(model_bytes / (avg_ms / 1000) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic_frac": None if traffic is None else round(traffic / (avg_ms / 1000) / 1e9 / HBM_PEAK_GBS, 4),
                "traffic_source": "rocprofv3 TCC_EA0_RDREQ_DRAM_32B_sum x 32 B + WRITE_SIZE x 1 KiB per dispatch "
                                  "(both exact on a 1 GiB copy), from profiles/" + (summary or "")}
    config = {"workload": f"triangle COUNT on R-MAT scale {args.scale}, 2^{args.samples_log2} samples "
                          f"(a=0.57,b=0.19,c=0.19), oriented low->high, set-mode dedup",
              "edges": n_edges, "wedges": wedges, "triangles": head["count"],
              "step": "trie_build + plan + join_aggregate + count readback",
              "policy": head_policy, "layout": head["layout"], "attr_order": head["order"],
              "join_kernels_ms_per_step": head["join_ms"], "protocol": head["protocol"]}
    if len(runs) == 2:
        pl = runs["plain"]
        config["plain"] = {"ms_per_step": pl["ms"], "tuples_per_s": pl["value"], "attr_order": pl["order"],
                           "layout": pl["layout"], "protocol": pl["protocol"]}
        config["learned_over_plain"] = round(pl["ms"] / head["ms"], 4)
        if head["protocol"]:
            config["learned_over_plain_cold"] = round(pl["protocol"]["cold"]["mean_drop_minmax_ms"]
                                                      / head["protocol"]["cold"]["mean_drop_minmax_ms"], 4)
    if not args.no_side:
        config["spgemm_4096"] = measure_spgemm(args, lh, torch, synth, flush)
        bat = measure_batch(args, lh, torch, synth)
        config["batch_512"] = bat
        config["learned_batched_over_plain_sequential"] = bat["learned_batched_over_plain_sequential"]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
    }
    del flush
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_scale, {"wedges": wedges, "edges": n_edges})
    print(json.dumps(out), flush=True)


def measure_triangle(args, lh, torch, lo_d, hi_d, layout, policy, flush):
    """Warm-up, then `steps` timed steps of trie build + plan + join + count
    readback under one layout and policy (kernels timed with HIP events on
    their stream); then the 7-run protocol, cold (caches flushed before each
    run) and warm."""
    state = {}

    def step():
        t = lh.trie_build([lo_d, hi_d], layout=layout)
        p = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count", policy=policy)
        r = lh.join_aggregate([p])[0]
        res = r.to_host()
        if "edges" not in state:
            state["edges"] = t.info()["level_size"][1]
            state["order"] = p.info()["attr_order"]
        state["count"] = int(res["counts"][0])
        r.free()
        p.free()
        t.free()

    for i in range(args.warmup):
        step()
        log(f"[{policy}] warmup {i}: triangles={state['count']} edges={state['edges']} order={state['order']}")
    torch.cuda.synchronize()
    lh.profile_reset()
    lh.profile_enable(True)
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lh.profile_enable(False)
    prof = lh.profile_read()
    protocol = None
    if args.runs:
        protocol = {"cold": run_protocol(torch, step, flush, args.runs), "warm": run_protocol(torch, step, None, args.runs)}
    gc.enable()
    ms = dt * 1000 / args.steps
    log(f"[{policy}] {args.steps} steps: {ms:.2f} ms/step, triangles={state['count']}; protocol {protocol}")
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"]):
        log(f"  {k:22s} launches={v['launches']:6d} total={v['total_ms']:9.3f} ms "
            f"rows={v['rows']} elems={v['elements']}")
    join_ms = sum(prof[k]["total_ms"] for k in prof if k.startswith(("join_", "leaf_"))) / args.steps
    return {"ms": ms, "value": 3 * state["edges"] / (ms / 1000), "prof": prof, "edges": state["edges"],
            "count": state["count"], "order": state["order"], "layout": layout, "join_ms": round(join_ms, 3),
            "protocol": protocol}


def measure_spgemm(args, lh, torch, synth, flush):
    """SpGEMM C(i,k) = SUM_j A(i,j) B(j,k), n = 4096, 10 distinct uniform
    columns per row, U(-1,1) values, order i,j,k: one step is both trie
    builds from resident columns + plan + join + readback.  Minimum bytes:
    both tries read once (4 B key + 4 B offset per entry level, 8 B value)
    and C written once (8 B of keys + 8 B count + 8 B sum per row)."""
    from tests import queries
    a = synth.sparse_matrix(4096, 10, seed=1)
    b = synth.sparse_matrix(4096, 10, seed=11)
    q = queries.spgemm(a, b)
    dev = [{"keys": [lh.to_device(k) for k in x["keys"]], "annos": [lh.to_device(v) for v in x["annos"]]}
           for x in q["atoms"]]
    state = {}

    def step():
        tries = [lh.trie_build(x["keys"], x["annos"], bag=True) for x in dev]
        p = lh.plan(3, [(tries[0], [0, 1], 0), (tries[1], [1, 2], 0)], out=[0, 2], agg="sum",
                    attr_order=[0, 1, 2], policy="fixed")
        r = lh.join_aggregate([p])[0]
        state["rows"] = r.n_rows
        state["products"] = int(r.to_host()["counts"].sum())
        r.free()
        p.free()
        for t in tries:
            t.free()

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000 / args.steps
    cold = run_protocol(torch, step, flush, args.runs) if args.runs else None
    nnz = len(a[0]) + len(b[0])
    alg = nnz * 16 + 2 * 4 * 4097 + state["rows"] * 24
    res = {"workload": "SpGEMM n = 4096, 10 nnz/row, order i,j,k (cfg1)", "ms_per_step": round(ms, 3),
           "tuples_per_s": nnz / (ms / 1000), "products": state["products"], "output_rows": state["rows"],
           "alg_bytes": alg, "alg_GBs": round(alg / (ms / 1000) / 1e9, 2),
           "frac": round(alg / (ms / 1000) / 1e9 / HBM_PEAK_GBS, 5), "protocol_cold": cold,
           "note": "a latency-bound step: the bytes fit on chip, so the fraction of HBM peak is not its bound"}
    log(f"spgemm 4096: {res}")
    return res


def measure_batch(args, lh, torch, synth):
    """The 512 SpMV / SpGEMM instances (n log-uniform in [1k, 64k], Zipf(1.1)
    row degrees with mean 16, U(-1,1) values), four ways: {plain rules,
    learned model} x {one lh_join_aggregate call per plan, one batched call
    (persistent kernels captured in a hipGraph, autotuned)}.  Tries and
    plans are built once, outside the timed region.  Every way must give the
    same results bit for bit.  Minimum bytes of one pass: per SpMV 12 B per
    nonzero + 4 B per row offset + 8 B per x and per y entry; per SpGEMM
    A(i,j) A(j,k) the trie read twice (12 B per nonzero + 4 B per row
    offset each time) and C written (8 B keys + 8 B count + 8 B sum per
    row)."""
    import hashlib
    log(f"generating {args.instances} instances")
    t0 = time.perf_counter()
    insts = synth.batched_instances(count=args.instances)
    log(f"  {sum(i['n'] for i in insts)} rows, {sum(len(i['rows']) for i in insts)} nonzeros "
        f"in {time.perf_counter() - t0:.1f} s")
    tuples = sum(len(i["rows"]) + i["n"] if i["kind"] == "spmv" else 2 * len(i["rows"]) for i in insts)
    dev = []
    for inst in insts:
        d = {"rows": lh.to_device(inst["rows"]), "cols": lh.to_device(inst["cols"]),
             "vals": lh.to_device(inst["vals"]), "n": inst["n"]}
        if inst["kind"] == "spmv":
            d["xk"] = lh.to_device(np.arange(inst["n"], dtype=np.uint32))
            d["x"] = lh.to_device(inst["x"])
        dev.append(d)
    del insts[:]

    def build(policy):
        layout = "learned" if policy == "learned" else "plain"
        tries, plans = [], []
        for d in dev:
            ta = lh.trie_build([d["rows"], d["cols"]], [d["vals"]], bag=True, layout=layout)
            tries.append(ta)
            if "x" in d:
                tx = lh.trie_build([d["xk"]], [d["x"]], bag=True, layout=layout)
                tries.append(tx)
                plans.append(lh.plan(2, [(ta, [0, 1], 0), (tx, [1], 0)], out=[0], agg="sum", policy=policy))
            else:
                plans.append(lh.plan(3, [(ta, [0, 1], 0), (ta, [1, 2], 0)], out=[0, 2], agg="sum", policy=policy))
        return tries, plans

    def digest(rs):
        h = hashlib.sha256()
        rows = 0
        for r in rs:
            o = r.to_host()
            rows += len(o["counts"])
            h.update(o["keys"].tobytes())
            h.update(o["counts"].tobytes())
            h.update(o["sums"].tobytes())
        return h.hexdigest(), rows

    legs, digests, orders = {}, {}, {}
    alg = None
    policies = [p for p in args.batch_policies.split(",") if p]
    for policy in policies:
        if policy == "learned":
            from paper_1708_07859_amd import learned as L
            lm, om, _ = L.load(args.weights or L.DEFAULT_WEIGHTS)
            L.register(lm, om)
        tries, plans = build(policy)
        orders[policy] = sorted({tuple(p.info()["attr_order"]) for p in plans})
        # sequential: one call per plan
        rs = [lh.join_aggregate([p])[0] for p in plans]
        digests[(policy, "sequential")] = digest(rs)
        if alg is None:
            alg = 0
            for d, r in zip(dev, rs):
                nnz = d["rows"].numel()
                n = d["n"]
                if "x" in d:
                    alg += 12 * nnz + 4 * (n + 1) + 16 * n
                else:
                    alg += 2 * (12 * nnz + 4 * (n + 1)) + 24 * r.n_rows
        for r in rs:
            r.free()
        torch.cuda.synchronize()
        if not args.no_sequential:
            gc.collect()
            gc.disable()
            seq = []
            for _ in range(max(1, args.steps // 2)):
                t0 = time.perf_counter()
                for p in plans:
                    lh.join_aggregate([p])[0].free()
                torch.cuda.synchronize()
                seq.append((time.perf_counter() - t0) * 1000)
            gc.enable()
            legs[(policy, "sequential")] = min(seq)
        # batched: the first call builds, tunes and captures; then replays
        t0 = time.perf_counter()
        rs = lh.join_aggregate(plans)
        first_s = time.perf_counter() - t0
        digests[(policy, "batched")] = digest(rs)
        for r in rs:
            r.free()
        for _ in range(args.warmup):
            for r in lh.join_aggregate(plans):
                r.free()
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        lh.profile_reset()
        lh.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for r in lh.join_aggregate(plans):
                r.free()
        torch.cuda.synchronize()
        legs[(policy, "batched")] = (time.perf_counter() - t0) * 1000 / args.steps
        lh.profile_enable(False)
        gc.enable()
        prof = lh.profile_read()
        log(f"[batch {policy}] orders {orders[policy]}; sequential {legs.get((policy, 'sequential'), 0):.1f} ms, "
            f"batched {legs[(policy, 'batched')]:.1f} ms (first call {first_s:.1f} s)")
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])[:8]:
            log(f"  {k:22s} launches={v['launches']:6d} total={v['total_ms']:9.3f} ms")
        for p in plans:
            p.free()
        for t in tries:
            t.free()
        if policy == "learned":
            lh.use_model(lh.LH_MODEL_LAYOUT, None)
            lh.use_model(lh.LH_MODEL_ORDER, None)
    assert len({d for d, _ in digests.values()}) == 1, "the ways disagree"
    if ("learned", "batched") not in legs or ("plain", "sequential") not in legs:
        res = {"workload": f"{args.instances} SpMV/SpGEMM instances (cfg4)",
               "ms": {f"{p}_{w}": round(v, 3) for (p, w), v in legs.items()},
               "tuples_per_s": {f"{p}_{w}": tuples / (v / 1000) for (p, w), v in legs.items()},
               "alg_bytes": alg, "input_tuples": tuples}
        log(f"batch: {res}")
        return res
    lb, ps = legs[("learned", "batched")], legs[("plain", "sequential")]
    res = {"workload": f"{args.instances} SpMV/SpGEMM instances, n log-uniform [1k,64k], Zipf(1.1) degrees "
                       "mean 16, FP64 U(-1,1) (cfg4)",
           "ms": {f"{p}_{w}": round(v, 3) for (p, w), v in legs.items()},
           "tuples_per_s": {f"{p}_{w}": tuples / (v / 1000) for (p, w), v in legs.items()},
           "learned_batched_over_plain_sequential": round(ps / lb, 4),
           "batched_over_sequential_plain": round(ps / legs[("plain", "batched")], 4),
           "orders": {k: [list(o) for o in v] for k, v in orders.items()},
           "output_rows": digests[("plain", "batched")][1], "input_tuples": tuples,
           "alg_bytes": alg, "alg_GBs_learned_batched": round(alg / (lb / 1000) / 1e9, 1),
           "frac_learned_batched": round(alg / (lb / 1000) / 1e9 / HBM_PEAK_GBS, 4),
           "sequential_timing": f"best of {max(1, args.steps // 2)} passes; batched: mean of {args.steps} replays"}
    log(f"batch: {res}")
    return res


def scope_roofline(prof, scope, steps):
    """GB/s and fraction of peak of one profiling scope whose `elements`
    field holds the algorithmic bytes its launches moved."""
    e = prof.get(scope)
    if not e or not e["total_ms"]:
        return None
    gbs = e["elements"] / (e["total_ms"] / 1000) / 1e9
    return {"kernel_scope": scope, "launches_per_step": e["launches"] / steps,
            "ms_per_step": round(e["total_ms"] / steps, 3), "bytes_per_step": int(e["elements"] / steps),
            "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def bench_configs(args, lh, torch, synth):
    """Every single-GPU configuration in one table: SpGEMM n = 4096 (cfg1),
    the triangle at 2^22 vertices (cfg2, the headline; see the default run),
    the 60M-row star GROUP BY (cfg3), the 512-instance batch (cfg4) and the
    held-out R-MAT 24 triangle (cfg5), each with tuples/s and the roofline
    fraction of its dominant kernel under a stated byte count."""
    from paper_1708_07859_amd import learned as L
    from tests import queries
    flush = torch.empty(FLUSH_BYTES, dtype=torch.uint8, device="cuda").zero_()
    table = {}
    table["cfg1"] = measure_spgemm(args, lh, torch, synth, flush)

    # cfg3: star join GROUP BY, one step = the five trie builds + plan + join
    log("generating the star schema")
    sch = synth.star_schema(seed=3)
    q = queries.star(sch)
    dev = [{"keys": [lh.to_device(k) for k in a["keys"]], "annos": [lh.to_device(x) for x in a.get("annos", [])],
            "meta": [lh.to_device(m) for m in a.get("meta", [])], "bag": a.get("bag", False)} for a in q["atoms"]]
    rows = sum(len(x["keys"][0]) for x in q["atoms"])
    del sch
    lm, om, _ = L.load(args.weights or L.DEFAULT_WEIGHTS)
    star = {}
    for policy in ("plain", "learned"):
        if policy == "learned":
            L.register(lm, om)
        layout = "learned" if policy == "learned" else "plain"
        state = {}

        def step():
            tries = [lh.trie_build(a["keys"], a["annos"], a["meta"], bag=a["bag"], layout=layout) for a in dev]
            atoms = [(t, a["attrs"], a.get("anno", -1)) for t, a in zip(tries, q["atoms"])]
            p = lh.plan(q["n_attrs"], atoms, out=q.get("out", []), group=q.get("group", []), agg=q["agg"],
                        filters=q.get("filters", []), policy=policy)
            state["order"] = p.info()["attr_order"]
            r = lh.join_aggregate([p])[0]
            o = r.to_host()
            state["groups"], state["tuples"] = len(o["counts"]), int(o["counts"].sum())
            r.free()
            p.free()
            for t in tries:
                t.free()

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        lh.profile_reset()
        lh.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / args.steps
        lh.profile_enable(False)
        prof = lh.profile_read()
        join_ms = sum(v["total_ms"] for k, v in prof.items() if k.startswith(("join_", "leaf_"))) / args.steps
        star[policy] = {"ms_per_step": round(ms, 3), "tuples_per_s": rows / (ms / 1000), "order": state["order"],
                        "groups": state["groups"], "join_tuples": state["tuples"],
                        "join_kernels_ms": round(join_ms, 3),
                        "roofline": scope_roofline(prof, "sort_scatter", args.steps),
                        "protocol_cold": run_protocol(torch, step, flush, args.runs) if args.runs else None}
        log(f"star {policy}: {star[policy]}")
        if policy == "learned":
            lh.use_model(lh.LH_MODEL_LAYOUT, None)
            lh.use_model(lh.LH_MODEL_ORDER, None)
    del dev
    table["cfg3"] = {"workload": "star join GROUP BY, 60M fact rows (Zipf 1.0 keys), dims 2M/500k/100k/10k, "
                                 "filters 20%/10%/1%, ~100 groups", "input_rows": rows,
                     "roofline_note": "dominant kernel: the radix-sort scatter of the trie builds, 16 B per key "
                                      "(24 B with a value) per pass",
                     **star}

    table["cfg4"] = measure_batch(args, lh, torch, synth)

    # cfg5: the held-out graph, both policies, every candidate for the regret
    log("generating R-MAT 24 (held out)")
    lo, hi = synth.rmat_edges(24, 1 << 28, seed=5)
    lo_d, hi_d = lh.to_device(lo), lh.to_device(hi)
    del lo, hi
    n_edges, wedges, _ = edge_stats(torch, lo_d, hi_d)
    b_min = triangle_min_bytes(n_edges, wedges, 1 << 24)

    def tri(layout, policy, order=None):
        torch.cuda.synchronize()
        lh.profile_reset()
        lh.profile_enable(True)
        t0 = time.perf_counter()
        t = lh.trie_build([lo_d, hi_d], layout=layout)
        p = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count", attr_order=order,
                    policy=policy)
        r = lh.join_aggregate([p])[0]
        c = int(r.to_host()["counts"][0])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000
        lh.profile_enable(False)
        prof = lh.profile_read()
        leaf = sum(v["total_ms"] for k, v in prof.items() if k in ("leaf_aggregate", "leaf_top"))
        chosen = p.info()["attr_order"]
        r.free()
        p.free()
        t.free()
        return ms, c, chosen, leaf

    def best(layout, policy, order=None, reps=3):
        rs = [tri(layout, policy, order) for _ in range(reps)]
        assert len({x[1] for x in rs}) == 1
        i = min(range(reps), key=lambda k: rs[k][0])
        return rs[i]

    L.register(lm, om)
    tri("plain", "plain")
    res5 = {}
    for policy in ("plain", "learned"):
        ms, c, chosen, leaf = best("learned" if policy == "learned" else "plain", policy)
        res5[policy] = {"ms_per_step": round(ms, 3), "tuples_per_s": 3 * n_edges / (ms / 1000), "order": chosen,
                        "leaf_ms": round(leaf, 3), "leaf_min_bytes_GBs": round(b_min / (leaf / 1000) / 1e9, 1),
                        "leaf_frac": round(b_min / (leaf / 1000) / 1e9 / HBM_PEAK_GBS, 4), "triangles": c}
    import itertools
    cands = {}
    for layout in ("plain", "learned"):
        for order in itertools.permutations(range(3)):
            ms, c, _, _ = best(layout, "fixed", list(order), reps=2)
            assert c == res5["plain"]["triangles"]
            cands[f"{layout}:{list(order)}"] = round(ms, 3)
    lh.use_model(lh.LH_MODEL_LAYOUT, None)
    lh.use_model(lh.LH_MODEL_ORDER, None)
    t_best = min(cands.values())
    assert res5["plain"]["triangles"] == res5["learned"]["triangles"]
    table["cfg5"] = {"workload": "held-out triangle COUNT, R-MAT scale 24, 2^28 samples, seed 5",
                     "edges": n_edges, "wedges": wedges, "leaf_min_bytes": b_min, **res5,
                     "speedup_learned_over_plain": round(res5["plain"]["ms_per_step"] / res5["learned"]["ms_per_step"], 4),
                     "regret_plain": round(res5["plain"]["ms_per_step"] / t_best - 1, 4),
                     "regret_learned": round(res5["learned"]["ms_per_step"] / t_best - 1, 4),
                     "candidates_ms": cands}
    out = {"metric": "per-configuration join-aggregate tuples/s and roofline fractions", "value": None,
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64",
           "data": "synthetic", "config": table}
    print(json.dumps(out), flush=True)


def bench_learned(args, lh, torch, synth):
    """Held-out evaluation of the learned cost model: triangle COUNT on an
    R-MAT graph it never saw (2^scale vertices, 2^(samples) samples).  Times
    a full step (trie build + plan + join) under the plain rule and under
    the learned policy, then every candidate (6 attribute orders x plain or
    learned layouts) for the regret of each policy."""
    import itertools

    from paper_1708_07859_amd import learned as L
    weights = args.weights or L.DEFAULT_WEIGHTS
    if os.path.exists(weights):
        lm, om, meta = L.load(weights)
        log(f"loaded {weights}")
    else:
        log("no trained weights: training now")
        Xl, yl, _ = L.calibrate_layouts()
        Xo, yo, _ = L.order_samples(L.training_queries())
        lm, _, _ = L.train_model(Xl, yl, lh.LH_LAYOUT_FEATURES)
        om, _, _ = L.train_model(Xo, yo, lh.LH_ORDER_FEATURES)
    log(f"generating R-MAT scale {args.scale}, 2^{args.samples_log2} samples (held out)")
    lo, hi = synth.rmat_edges(args.scale, 1 << args.samples_log2, seed=5)
    lo_d, hi_d = lh.to_device(lo), lh.to_device(hi)
    del lo, hi

    def run(layout, policy, order=None):
        torch.cuda.synchronize()
        lh.profile_reset()
        lh.profile_enable(True)
        t0 = time.perf_counter()
        t = lh.trie_build([lo_d, hi_d], layout=layout)
        p = lh.plan(3, [(t, [0, 1], -1), (t, [1, 2], -1), (t, [0, 2], -1)], agg="count", attr_order=order,
                    policy=policy)
        r = lh.join_aggregate([p])[0]
        c = int(r.to_host()["counts"][0])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1000
        lh.profile_enable(False)
        prof = lh.profile_read()
        build = sum(v["total_ms"] for k, v in prof.items() if k.startswith(("trie_", "sort_", "layout")))
        join = sum(v["total_ms"] for k, v in prof.items() if k.startswith(("join_", "leaf_")))
        chosen = p.info()["attr_order"]
        words = sum(t.info()["level_words"])
        log(f"    {layout:7s} {policy:7s} {str(chosen):9s} {dt:8.1f} ms (build kernels {build:.1f}, join kernels "
            f"{join:.1f}, bitset words {words})")
        r.free()
        p.free()
        t.free()
        return dt, c, chosen

    def best_of(layout, policy, order=None, reps=2):
        res = [run(layout, policy, order) for _ in range(reps)]
        return min(r[0] for r in res), res[0][1], res[0][2]

    L.register(lm, om)
    run("plain", "plain")                                   # warm-up
    t_plain, c_plain, o_plain = best_of("plain", "plain")
    t_learn, c_learn, o_learn = best_of("learned", "learned")
    log(f"plain {t_plain:.1f} ms order {o_plain}; learned {t_learn:.1f} ms order {o_learn}")
    assert c_plain == c_learn, (c_plain, c_learn)
    cands = {}
    for layout in ("plain", "learned"):
        for order in itertools.permutations(range(3)):
            t, c, _ = best_of(layout, "fixed", list(order), reps=2)
            assert c == c_plain
            cands[f"{layout}:{list(order)}"] = t
            log(f"  candidate {layout} {list(order)}: {t:.1f} ms")
    best = min(cands.values())
    out = {
        "metric": METRIC, "value": t_plain / t_learn, "unit": "speedup (plain / learned)", "n_gpus": 1,
        "steps": 2, "warmup": 1, "ms_per_step": t_learn, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"held-out triangle COUNT, R-MAT scale {args.scale}, 2^{args.samples_log2} samples, "
                               "seed 5", "triangles": c_plain,
                   "plain_ms": t_plain, "learned_ms": t_learn, "plain_order": o_plain, "learned_order": o_learn,
                   "regret_plain": t_plain / best - 1, "regret_learned": t_learn / best - 1,
                   "best_candidate_ms": best, "candidates_ms": cands},
    }
    print(json.dumps(out), flush=True)


def bench_intersect(args, lh, torch, synth):
    """Set-pair intersections, the shape of the paper's intersection
    micro-benchmark (Fig. 5a, section 6.3): `pairs` pairs of sets of `card`
    elements drawn without replacement from [0, 2*card) (density 1/2),
    intersected as R(p,x) |x| S(p,x) COUNT GROUP BY p in one launch, with the
    sets as uint arrays or bitsets; plus a sparse variant (universe 64*card,
    uint arrays).  Algorithmic bytes per pair: uint & uint 8c (both sets
    streamed), uint & bitset 4c + U/8, bitset & bitset 2 U/8 (U = universe)."""
    import numpy as np
    c, npairs = args.card, args.pairs
    variants = [("uint", "uint", 2), ("uint", "bitset", 2), ("bitset", "bitset", 2), ("uint", "uint", 64)]
    results = {}
    pairs_of = {}
    for la, lb, mult in variants:
        U = mult * c
        if U not in pairs_of:
            log(f"generating {npairs} pairs of {c} elements from [0, {U})")
            t0 = time.perf_counter()
            pairs = synth.set_pairs(c, U, npairs, seed=100 if mult == 2 else 101)
            pr = np.repeat(np.arange(npairs, dtype=np.uint32), c)
            xr = np.concatenate([a for a, _ in pairs])
            xs = np.concatenate([b for _, b in pairs])
            want = [len(np.intersect1d(pairs[i][0], pairs[i][1], assume_unique=True)) for i in range(0, npairs,
                                                                                                  max(1, npairs // 8))]
            pairs_of[U] = (lh.to_device(pr), lh.to_device(xr), lh.to_device(xs), want)
            del pairs, pr, xr, xs
            log(f"  {time.perf_counter() - t0:.1f} s")
        pr_d, xr_d, xs_d, want = pairs_of[U]
        ta = lh.trie_build([pr_d, xr_d], layout=la)
        tb = lh.trie_build([pr_d, xs_d], layout=lb)
        p = lh.plan(2, [(ta, [0, 1], -1), (tb, [0, 1], -1)], out=[0], agg="count", attr_order=[0, 1],
                    policy="fixed")
        for _ in range(max(1, args.warmup)):
            r = lh.join_aggregate([p])[0]
            res = r.to_host()
            r.free()
        got = res["counts"][::max(1, npairs // 8)].tolist()
        assert got == want, (got, want)
        torch.cuda.synchronize()
        lh.profile_reset()
        lh.profile_enable(True)
        for _ in range(args.steps):
            lh.join_aggregate([p])[0].free()
        torch.cuda.synchronize()
        lh.profile_enable(False)
        prof = lh.profile_read()
        # the leaf: its main launch, the top-bucket launch (pairs of 2^14
        # elements or more) and the merge launch (two sorted sets of 2^12
        # elements or more, sizes within a factor of 4)
        ms = sum(prof[k]["total_ms"] for k in LEAF_SCOPES if k in prof) / args.steps
        per_pair = {("uint", "uint"): 8 * c, ("uint", "bitset"): 4 * c + U / 8,
                    ("bitset", "bitset"): 2 * U / 8}[(la, lb)]
        alg = per_pair * npairs
        gbs = alg / (ms / 1000) / 1e9
        name = f"{la}&{lb} density 1/{mult}"
        results[name] = {"leaf_ms": round(ms, 4), "alg_bytes": int(alg), "achieved_GBs": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "elements_per_s": 2 * c * npairs / (ms / 1000),
                         "units_ms": round(prof.get("leaf_units", {"total_ms": 0, "launches": 1})["total_ms"]
                                           / max(1, prof.get("leaf_units", {"launches": 1})["launches"]), 4)}
        log(f"{name}: leaf {ms:.3f} ms, {gbs:.0f} GB/s algorithmic ({gbs / HBM_PEAK_GBS:.1%} of peak)")
        p.free()
        ta.free()
        tb.free()
    head = results["uint&uint density 1/2"]
    out = {"metric": "set-pair intersection, algorithmic HBM GB/s of the leaf kernel", "value": head["achieved_GBs"],
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["leaf_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"{npairs} set pairs of {c} elements, COUNT of each intersection",
                      "variants": results}}
    print(json.dumps(out), flush=True)


def bench_q5(args, lh, torch, synth):
    """Multi-node plans (sections 2.3, 3.2) on the Q5-shaped schema at scale
    factor `sf`: SUM(lineitem.ann) GROUP BY nation over the customer /
    orders / lineitem / supplier cycle and the nation / region tail, with an
    equality selection on region and a one-year range on orders.  One step
    builds the six tries from resident columns, then runs the query; the
    decompositions timed are the library's choice, one generic-join node
    (width 3), the same two nodes with the tail as root (the last tie-break
    reversed) and the tail split into a chain (more nodes and depth, same
    width); the chosen plan runs once with the plain rule's attribute orders
    in every node and once with the learned model's.  value = input rows /
    step time of the chosen plan under the learned orders (the plain
    rule's time sits in the config)."""
    import numpy as np

    from tests import queries
    log(f"generating the Q5-shaped schema at sf {args.sf}")
    sch = synth.q5_schema(args.sf, seed=5)
    q = queries.q5(sch)
    dev = [{"keys": [lh.to_device(k) for k in a["keys"]], "annos": [lh.to_device(x) for x in a.get("annos", [])],
            "meta": [lh.to_device(m) for m in a.get("meta", [])], "bag": a.get("bag", False)} for a in q["atoms"]]
    n_rows = sum(len(a["keys"][0]) for a in q["atoms"])
    del sch
    args_q = dict(out=q["out"], agg="sum", filters=q["filters"])
    from paper_1708_07859_amd import learned as L
    weights = args.weights or L.DEFAULT_WEIGHTS
    lm, om, _ = L.load(weights)
    L.register(lm, om)
    variants = {
        "chosen": (None, "plain"),
        "chosen, learned orders": (None, "learned"),
        "one node": ("single", "plain"),
        "tail as root": ({"edges": [0b110000, 0b001111], "parent": [-1, 0], "pushed": [0, 0]}, "plain"),
        "chain tail": ({"edges": [0b001111, 0b010000, 0b100000], "parent": [-1, 0, 1], "pushed": [0, 0, 0]}, "plain"),
    }

    def step(g, policy):
        tries = [lh.trie_build(a["keys"], a["annos"], a["meta"], bag=a["bag"]) for a in dev]
        atoms = [(t, a["attrs"], a.get("anno", -1)) for t, a in zip(tries, q["atoms"])]
        if g == "single":
            p = lh.plan(q["n_attrs"], atoms, policy=policy, **args_q)
            r = lh.join_aggregate([p])[0]
            out = r.to_host()
            r.free()
            p.free()
        else:
            r = lh.ghd_join_aggregate(q["n_attrs"], atoms, ghd=g, policy=policy, **args_q)
            out = r.to_host()
            r.free()
        chosen = lh.ghd_for_query(q["n_attrs"], atoms, **args_q) if g is None else None
        for t in tries:
            t.free()
        return out, chosen

    results, ref, chosen = {}, None, None
    for name, (g, policy) in variants.items():
        for _ in range(max(1, args.warmup)):
            out, ch = step(g, policy)
            chosen = ch or chosen
        if ref is None:
            ref = out
        assert np.array_equal(out["keys"], ref["keys"]) and np.array_equal(out["counts"], ref["counts"])
        assert np.all(np.abs(out["sums"] - ref["sums"]) <= 1e-9 * np.abs(ref["sums"]))
        torch.cuda.synchronize()
        if name.startswith("chosen"):
            lh.profile_reset()
            lh.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(g, policy)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / args.steps
        if name.startswith("chosen"):
            lh.profile_enable(False)
            prof = lh.profile_read()
            log(f"{name}, top scopes:")
            top = sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])[:12]
            for k, v in top:
                log(f"  {k:22s} {v['total_ms'] / args.steps:8.2f} ms/step  launches {v['launches'] // args.steps}")
        results[name] = {"ms_per_step": round(ms, 3), "rows_per_s": n_rows / (ms / 1000)}
        log(f"{name}: {ms:.2f} ms/step")
    head = results["chosen, learned orders"]
    out = {"metric": "join-aggregate input tuples/s, multi-node plan", "value": head["rows_per_s"],
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32+f64", "data": "synthetic",
           "config": {"workload": f"Q5-shaped SUM GROUP BY nation, sf {args.sf}, {n_rows} input rows",
                      "step": "6 x trie_build + GHD plan + join_aggregate per node + readback",
                      "groups": len(ref["counts"]), "join_tuples": ref["n_join"],
                      "ghd": {"edges": chosen["edges"], "parent": chosen["parent"], "pushed": chosen["pushed"],
                              "fhw": chosen["fhw"]},
                      "variants": results,
                      "chosen_over_one_node": results["one node"]["ms_per_step"] / head["ms_per_step"]}}
    print(json.dumps(out), flush=True)


def bench_groupby(args, lh, torch, synth):
    """GROUP BY implementations (section 5, Fig. 6 shapes).

    Key union: R(x,y) |x| S(y,z), SUM(R.v * S.w) GROUP BY z under the order
    x,y,z, so the leaf's z values are unioned by a GROUP BY; about 10^7 join
    tuples; z drawn from a random subset of [0, 10^6) whose size sets the
    output density (Fig. 6a).  Wide key: the same join grouped by x, z and
    three meta columns (a five-value key, Fig. 6c) with about 10^6 groups.
    Each implementation runs the same plan; only lh_join_aggregate is
    timed."""
    import numpy as np

    rng = synth.rng_for(31)
    n_r, n_s, dom_x, dom_y, zr = 10_000, 1_000_000, 1000, 1000, 1_000_000
    rx = rng.integers(0, dom_x, n_r).astype(np.uint32)
    ry = rng.integers(0, dom_y, n_r).astype(np.uint32)
    rv = rng.integers(-8, 9, n_r) / 8.0
    sy = rng.integers(0, dom_y, n_s).astype(np.uint32)
    sw = synth.uniform_pm1(rng, n_s)
    rm = [rng.integers(0, 16, n_r).astype(np.uint32), rng.integers(0, 64, n_r).astype(np.uint32)]
    sm = [rng.integers(0, 8, n_s).astype(np.uint32)]
    tr = lh.trie_build([lh.to_device(rx), lh.to_device(ry)], [lh.to_device(rv)], [lh.to_device(m) for m in rm],
                       bag=True)
    impls = ["sort", "hash", "dense", "auto"]

    def time_plan(p):
        for _ in range(max(1, args.warmup)):
            r = lh.join_aggregate([p])[0]
            out = r.to_host()
            r.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lh.join_aggregate([p])[0].free()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000 / args.steps, out

    sweep = {}
    for density in [1e-4, 1e-3, 1e-2, 1e-1, 1.0]:
        values = rng.choice(zr, max(1, int(density * zr)), replace=False).astype(np.uint32)
        sz = values[rng.integers(0, len(values), n_s)]
        ts = lh.trie_build([lh.to_device(sy), lh.to_device(sz)], [lh.to_device(sw)], bag=True)
        row, ref = {}, None
        for impl in impls:
            p = lh.plan(3, [(tr, [0, 1], 0), (ts, [1, 2], 0)], out=[2], agg="sum", attr_order=[0, 1, 2],
                        policy="fixed", group_impl=impl)
            ms, out = time_plan(p)
            p.free()
            if ref is None:
                ref = out
            assert np.array_equal(out["keys"], ref["keys"]) and np.array_equal(out["counts"], ref["counts"])
            assert np.array_equal(out["sums"].view(np.uint64), ref["sums"].view(np.uint64))
            row[impl] = round(ms, 3)
            if impl == "auto":
                row["auto_chose"] = out["group_impl"]
        row["groups"] = len(ref["counts"])
        row["join_tuples"] = int(ref["counts"].sum())
        sweep[f"density {density:g}"] = row
        log(f"key union, output density {density:g}: {row}")
        ts.free()
    # wide key
    sz = rng.integers(0, 4096, n_s).astype(np.uint32)
    ts = lh.trie_build([lh.to_device(sy), lh.to_device(sz)], [lh.to_device(sw)], [lh.to_device(sm[0])], bag=True)
    wide, ref = {}, None
    for impl in ["sort", "hash", "auto"]:
        p = lh.plan(3, [(tr, [0, 1], 0), (ts, [1, 2], 0)], out=[0, 2], group=[(0, 0), (0, 1), (1, 0)], agg="sum",
                    attr_order=[0, 1, 2], policy="fixed", group_impl=impl)
        ms, out = time_plan(p)
        p.free()
        if ref is None:
            ref = out
        assert np.array_equal(out["keys"], ref["keys"]) and np.array_equal(out["counts"], ref["counts"])
        wide[impl] = round(ms, 3)
        if impl == "auto":
            wide["auto_chose"] = out["group_impl"]
    wide["groups"] = len(ref["counts"])
    wide["join_tuples"] = int(ref["counts"].sum())
    log(f"wide key (5 values): {wide}")
    ts.free()
    tr.free()
    head = sweep["density 0.01"]
    out = {"metric": "join-aggregate tuples/s, GROUP BY outside the order's prefix", "unit": "tuples/s",
           "value": head["join_tuples"] / (head["auto"] / 1000), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["auto"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32+f64", "data": "synthetic",
           "config": {"workload": "R(x,y) join S(y,z), SUM GROUP BY z under order x,y,z; 10^4 x 10^6 rows, "
                                  "about 10^7 join tuples; z from a subset of [0, 10^6)",
                      "key_union_ms": sweep, "wide_key_ms": wide}}
    print(json.dumps(out), flush=True)


def bench_dense(args, lh, torch, synth):
    """Dense LA by attribute elimination (Table 3's DMV and DMM, n = 16384):
    completely dense relations A(i,j), B(j,k) / x(j) with U(-1,1) values.
    Times lh_join_aggregate of the planned query with LH_DENSE_BLAS (rocBLAS
    DGEMV / DGEMM over the annotation buffers, plus the output key columns)
    and, where it finishes in seconds, the exact generic join of the same
    query.  Roofline: DGEMM against the 78.6 TFLOP/s FP64 matrix peak
    (2 n^3 flops), DGEMV against 8 TB/s (8 n^2 bytes of matrix)."""
    import numpy as np

    def dense_trie(rows, cols, seed):
        rng = synth.rng_for(seed)
        r = torch.arange(rows, dtype=torch.int64, device="cuda").repeat_interleave(cols).to(torch.int32)
        c = torch.arange(cols, dtype=torch.int64, device="cuda").repeat(rows).to(torch.int32)
        v = torch.from_numpy(synth.uniform_pm1(rng, rows * cols)).cuda()
        t = lh.trie_build([r, c], [v], bag=True)
        del r, c, v
        return t

    def timed(p, steps):
        r = lh.join_aggregate([p])[0]
        r.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lh.join_aggregate([p])[0].free()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000 / steps

    res = {}
    for n, exact_too in [(1024, True), (4096, False), (16384, False)]:
        log(f"DMM n={n}")
        ta = dense_trie(n, n, 1)
        tb = dense_trie(n, n, 2)
        atoms = [(ta, [0, 1], 0), (tb, [1, 2], 0)]
        p = lh.plan(3, atoms, out=[0, 2], agg="sum", dense_blas=True)
        assert p.info()["blas"] == 2
        ms = timed(p, max(1, args.steps))
        p.free()
        row = {"blas_ms": round(ms, 3), "tflops": round(2 * n ** 3 / (ms / 1000) / 1e12, 2)}
        if exact_too:
            p = lh.plan(3, atoms, out=[0, 2], agg="sum")
            row["exact_join_ms"] = round(timed(p, 1), 3)
            p.free()
        res[f"DMM {n}"] = row
        log(f"  {row}")
        ta.free()
        tb.free()
    for n, exact_too in [(16384, True)]:
        log(f"DMV n={n}")
        tm = dense_trie(n, n, 3)
        x = torch.from_numpy(synth.uniform_pm1(synth.rng_for(4), n)).cuda()
        tx = lh.trie_build([torch.arange(n, dtype=torch.int32, device="cuda")], [x], bag=True)
        atoms = [(tm, [0, 1], 0), (tx, [1], 0)]
        p = lh.plan(2, atoms, out=[0], agg="sum", dense_blas=True)
        assert p.info()["blas"] == 1
        ms = timed(p, max(1, args.steps))
        p.free()
        row = {"blas_ms": round(ms, 3), "GBs": round(8 * n * n / (ms / 1000) / 1e9, 1)}
        if exact_too:
            p = lh.plan(2, atoms, out=[0], agg="sum")
            row["exact_join_ms"] = round(timed(p, 2), 3)
            p.free()
        res[f"DMV {n}"] = row
        log(f"  {row}")
        tm.free()
        tx.free()
    head = res["DMM 16384"]
    out = {"metric": "dense LA via attribute elimination, FP64 TFLOP/s of DMM n=16384", "value": head["tflops"],
           "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": head["blas_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "completely dense A(i,j), B(j,k), x(j), U(-1,1) values",
                      "results": res,
                      "roofline": {"bound": "mfma", "achieved": head["tflops"], "peak": 78.6, "unit": "TFLOP/s",
                                   "frac": round(head["tflops"] / 78.6, 4)}}}
    print(json.dumps(out), flush=True)


def bench_spgemm_star(args, lh, torch, synth):
    """The two other single-GPU workloads, timed as full steps (trie builds
    from resident columns + plan + join + readback):
    SpGEMM C(i,k) = SUM_j A(i,j) * A'(j,k), n = 4096, 10 distinct uniform
    columns per row, U(-1,1) values, attribute order i,j,k; and the star
    join with GROUP BY on 60M fact rows (Zipf 1.0 keys, dims of 2M / 500k /
    100k / 10k rows, filters of 20% / 10% / 1%), under the plain rule and
    the learned model."""
    from paper_1708_07859_amd import learned as L
    from tests import queries
    lm, om, _ = L.load(args.weights or L.DEFAULT_WEIGHTS)
    L.register(lm, om)

    def devq(q):
        return [{"keys": [lh.to_device(k) for k in a["keys"]],
                 "annos": [lh.to_device(x) for x in a.get("annos", [])],
                 "meta": [lh.to_device(m) for m in a.get("meta", [])], "bag": a.get("bag", False)}
                for a in q["atoms"]]

    def timed(q, dev, **kw):
        def step():
            tries = [lh.trie_build(a["keys"], a["annos"], a["meta"], bag=a["bag"]) for a in dev]
            atoms = [(t, a["attrs"], a.get("anno", -1)) for t, a in zip(tries, q["atoms"])]
            p = lh.plan(q["n_attrs"], atoms, out=q.get("out", []), group=q.get("group", []), agg=q["agg"],
                        filters=q.get("filters", []), **kw)
            r = lh.join_aggregate([p])[0]
            out = r.to_host()
            r.free()
            p.free()
            for t in tries:
                t.free()
            return out
        for _ in range(max(1, args.warmup)):
            out = step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000 / args.steps, out

    res = {}
    a = synth.sparse_matrix(4096, 10, seed=1)
    b = synth.sparse_matrix(4096, 10, seed=11)
    q = queries.spgemm(a, b)
    ms, out = timed(q, devq(q), attr_order=[0, 1, 2], policy="fixed")
    res["spgemm 4096, order i,j,k"] = {"ms_per_step": round(ms, 3), "output_rows": len(out["counts"]),
                                       "products": int(out["counts"].sum()),
                                       "products_per_s": int(out["counts"].sum()) / (ms / 1000)}
    log(f"spgemm: {res['spgemm 4096, order i,j,k']}")
    sch = synth.star_schema()
    q = queries.star(sch)
    dev = devq(q)
    del sch
    rows = sum(len(x["keys"][0]) for x in q["atoms"])
    for policy in ("plain", "learned"):
        ms, out = timed(q, dev, policy=policy)
        res[f"star 60M, {policy}"] = {"ms_per_step": round(ms, 3), "groups": len(out["counts"]),
                                      "join_tuples": int(out["counts"].sum()), "input_rows": rows,
                                      "rows_per_s": rows / (ms / 1000)}
        log(f"star {policy}: {res[f'star 60M, {policy}']}")
    head = res["star 60M, learned"]
    out = {"metric": "join-aggregate input tuples/s, star GROUP BY and SpGEMM", "value": head["rows_per_s"],
           "unit": "tuples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32+f64", "data": "synthetic",
           "config": {"workload": "star join GROUP BY on 60M fact rows; SpGEMM n = 4096", "results": res}}
    print(json.dumps(out), flush=True)


def bench_voter(args, lh, torch, synth):
    """The voter classification application of section 7 on synthetic
    tables of its sizes (7,503,555 voters, 2,751 precincts): the filtered
    join, the categorical encoding of its result, the design matrix's two
    tries and five iterations of logistic regression on them.  The base
    tables' tries are resident before the timed region (loaded data); every
    step runs the whole application.  Roofline: the two training kernels
    against HBM, with algorithmic bytes per launch
      lr_rows: nnz * (4 B feature + 8 B value) + n * (4 B row + 4 B offset + 8 B label + 8 B residual)
      lr_cols_blocked (row-id blocks of 4096): nnz * (4 B row + 8 B value) + n_ids * 8 B residual
                      + features * blocks * 8 B partial sums
      lr_cols (chunks of 2048 entries): nnz * (4 B row + 8 B value + 8 B residual gather) + chunks * 8 B."""
    import numpy as np

    from paper_1708_07859_amd import pipeline

    log(f"voter tables: {args.voters} voters, 2751 precincts")
    d = synth.voter_schema(args.voters, 2751, seed=7)
    feats = synth.voter_features(d)
    t = pipeline.VoterTables(d, feats)
    torch.cuda.synchronize()
    f = synth.VOTER_FILTER
    for _ in range(max(1, args.warmup)):
        out = pipeline.run(t, iters=5, step=0.5, **f)
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = pipeline.run(t, iters=5, step=0.5, **f)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000 / args.steps
    gc.enable()
    n_rows, nf = out["n_rows"], out["n_feat"]
    loss = out["loss"].cpu().numpy().tolist()
    log(f"  {ms:.2f} ms per pipeline; {n_rows} rows x {nf} features; loss {loss}")

    # kernel scopes of one whole pipeline
    lh.profile_reset()
    lh.profile_enable(True)
    pipeline.run(t, iters=5, step=0.5, **f)
    torch.cuda.synchronize()
    lh.profile_enable(False)
    for k, v in sorted(lh.profile_read().items(), key=lambda kv: -kv[1]["total_ms"])[:14]:
        log(f"  {k:22s} launches={v['launches']:5d} total={v['total_ms']:8.3f} ms")
    # phase split (one extra run, synchronised between phases)
    phases = {}
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    res = pipeline.sql_phase(t, **f)
    torch.cuda.synchronize()
    c1 = time.perf_counter()
    rows, fe, vals, _ = lh.encode(res.key_columns(), 0, t.features)
    torch.cuda.synchronize()
    c2 = time.perf_counter()
    res.free()
    xr, xc = pipeline.design_tries(rows, fe, vals)
    torch.cuda.synchronize()
    c3 = time.perf_counter()
    del rows, fe, vals
    w = torch.zeros(nf, dtype=torch.float64, device="cuda")
    lh.logreg_fit(xr, xc, t.y, w, 5, 0.5)
    torch.cuda.synchronize()
    c4 = time.perf_counter()
    phases = {"sql_ms": round((c1 - c0) * 1000, 3), "encode_ms": round((c2 - c1) * 1000, 3),
              "design_tries_ms": round((c3 - c2) * 1000, 3), "logreg_5_iters_ms": round((c4 - c3) * 1000, 3)}
    log(f"  phases {phases}")
    nnz = xr.info()["level_size"][1]
    n0 = xr.info()["level_size"][0]
    # kernel times of the training loop, on the stream the kernels run on
    lh.profile_reset()
    lh.profile_enable(True)
    w = torch.zeros(nf, dtype=torch.float64, device="cuda")
    lh.logreg_fit(xr, xc, t.y, w, 5, 0.5)
    torch.cuda.synchronize()
    lh.profile_enable(False)
    prof = lh.profile_read()
    _, foffs = xc.read_level(0)
    chunks = int(np.sum((np.diff(foffs.astype(np.int64)) + 2047) // 2048))
    rk, _ = xr.read_level(0)
    n_ids = int(rk[-1]) + 1 if len(rk) else 0
    blocks = (n_ids + 4095) // 4096
    xr.free()
    xc.free()
    t.free()
    alg = {"lr_rows": nnz * 12 + n0 * 24, "lr_cols": nnz * 20 + chunks * 8,
           "lr_cols_blocked": nnz * 12 + n_ids * 8 + (len(foffs) - 1) * blocks * 8}
    kern = {}
    for k, b in alg.items():
        e = prof.get(k)
        if e and e["launches"]:
            avg = e["total_ms"] / e["launches"]
            kern[k] = {"avg_ms": round(avg, 4), "alg_bytes": int(b), "GBs": round(b / (avg / 1000) / 1e9, 1)}
    log(f"  kernels {kern}")
    dom = max(kern, key=lambda k: kern[k]["avg_ms"]) if kern else None
    roof = None
    if dom:
        traffic = None
        if args.voters == 7_503_555:
            from paper_1708_07859_amd import profiling
            traffic = profiling.read_traffic(os.path.join(ROOT, "profiles", f"voter_{dom}_traffic.txt"), "k_" + dom)
        roof = {"kernel": "k_" + dom, "bound": "hbm", "achieved": kern[dom]["GBs"], "peak": 8000.0, "unit": "GB/s",
                "frac": round(kern[dom]["GBs"] / 8000.0, 4), "traffic": None if traffic is None else int(traffic),
                "avg_launch_ms": kern[dom]["avg_ms"], "alg_bytes_per_launch": kern[dom]["alg_bytes"]}

    cpu = None
    if not args.no_cpu:
        from oracle import ml
        m = args.voters
        ds = d
        c0 = time.perf_counter()
        vid, pid = ml.sql_phase(ds["voters"], ds["precincts"], **f)
        r_, f_, v_, nf_ = ml.encode([vid, pid], 0, synth.voter_features(ds))
        row_ids, X = ml.design_matrix(r_, f_, v_, nf_)
        ml.logreg(X, ds["voters"]["voted"][row_ids], np.zeros(nf_), 5, 0.5)
        sec = time.perf_counter() - c0
        cpu = {"value": round(m / sec, 1), "unit": "voters/s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": f"the whole workload ({m} voters), the same pipeline with a dense design matrix, "
                         f"{sec:.1f} s"}
        log(f"  cpu oracle {cpu}")
    value = args.voters / (ms / 1000)
    outj = {"metric": "voter classification pipeline (SQL + encoding + 5 logistic regression iterations), voters/s",
            "value": round(value, 1), "unit": "voters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"voter classification, {args.voters} voters x 2751 precincts, "
                                   f"{n_rows} selected rows, {nf} features, {nnz} design-matrix entries",
                       "phases": phases, "kernels": kern},
            "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(outj), flush=True)


def bench_copy(args, torch):
    """A plain device-to-device copy of 1 GiB: the known-size kernel that
    hardware byte counters (FETCH_SIZE, WRITE_SIZE) are scaled against, and
    the achievable-bandwidth line next to the 8 TB/s peak."""
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gbs = 2 * n / (ms / 1000) / 1e9
    out = {"metric": "device copy GB/s (read + write)", "value": gbs, "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "copy of 1 GiB, device to device", "bytes_read": n, "bytes_written": n,
                      "frac_of_peak": gbs / HBM_PEAK_GBS}}
    print(json.dumps(out), flush=True)


def bench_batch(args, lh, torch, synth):
    """The batched workload on its own: the four ways of measure_batch,
    reported as the learned + batched throughput."""
    res = measure_batch(args, lh, torch, synth)
    if "learned_batched_over_plain_sequential" not in res:
        key = next(k for k in res["ms"] if k.endswith("batched"))
        print(json.dumps({"metric": METRIC, "value": res["tuples_per_s"][key], "unit": "tuples/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms"][key],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": res}), flush=True)
        return
    lb = res["ms"]["learned_batched"]
    out = {
        "metric": METRIC, "value": res["tuples_per_s"]["learned_batched"], "unit": "tuples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": lb, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": res,
        "roofline": {"bound": "hbm", "kernel": "batched graph launch (all kernels)",
                     "achieved": res["alg_GBs_learned_batched"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": res["frac_learned_batched"], "traffic": None},
    }
    print(json.dumps(out), flush=True)


def bench_gather(args, torch):
    """Random 64-byte lines gathered from a 4 GiB array into a contiguous
    output: a kernel of known size whose reads are single 64-byte lines at
    random places, the access shape of set probes, next to the streaming
    copy.  Reads 64 B per line + 8 B per index, writes 64 B per line."""
    n_src = (4 << 30) // 64
    n_idx = 1 << 24
    src = torch.empty((n_src, 16), dtype=torch.int32, device="cuda").fill_(1)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    idx = torch.randint(0, n_src, (n_idx,), device="cuda", generator=g)
    out = torch.empty((n_idx, 16), dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        torch.index_select(src, 0, idx, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        torch.index_select(src, 0, idx, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    read, written = n_idx * 64 + n_idx * 8, n_idx * 64
    gbs = (read + written) / (ms / 1000) / 1e9
    print(json.dumps({"metric": "random 64-byte line gather GB/s (read + write)", "value": gbs, "unit": "GB/s",
                      "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32",
                      "data": "synthetic",
                      "config": {"workload": f"gather of {n_idx} random 64-byte lines from 4 GiB",
                                 "bytes_read": read, "bytes_written": written,
                                 "frac_of_peak": gbs / HBM_PEAK_GBS}}), flush=True)


if __name__ == "__main__":
    main()
