"""Benchmark of the BMLP hot path on one MI355X.

Workload (one "step"): the n = 16,384 directed Erdos-Renyi density sweep,
p in {1e-4, 5e-4, 1e-3, 5e-3, 1e-2} (seeded synthetic graphs shaped like the
paper's DG / DG+partial benchmarks).  For each of the five graphs a step
  1. packs the device-resident COO edge list into the n x n bit matrix,
  2. computes the full closure R1+ with BMLP-RMS (all n groundings r2(X, Y)),
  3. answers SMP queries r2(c, Y) from 1, 64 and 1,024 sources.
Inputs are resident in HBM before the timed region, and the timed steps ask
for no statistics.  The value is answered query rows per second (a closure
answers n rows; an SMP batch answers k).

Also reported: the live roofline of the dominant kernel (the matrix-core
product), measured in instrumented steps after the timed region with HIP events
around each product launch on the stream it runs on, and the CPU oracle timed
on a bounded sample of the same workload on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peaks in Boolean operations per second (one AND + one OR per bit-MAC, like the 2 flops of an FMA):
# VALU: 256 CUs x 64 lanes x 2.4 GHz x 32 bits x 2 ops (one v_and_or_b32 = 32 ANDs + 32 ORs);
# matrix cores: the published dense rate of the 4-bit (fp4 / e2m1) format the product kernel feeds them,
# 10.1 POPS (2 ops per multiply-accumulate).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 * 32 * 2 / 1e12
MFMA_FP4_PEAK_TOPS = 10.1e15 / 1e12
KERNELS = {0: ("k_gemm_valu", "bit-packed Boolean product on the VALU", "alu", VALU_PEAK_TOPS),
           1: ("k_gemm_mfma", "Boolean product on 4-bit (e2m1) matrix cores, exact fp32 count > 0", "mfma",
               MFMA_FP4_PEAK_TOPS)}

# HBM bytes per launch of the product kernels on this workload: rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch) scaled by the same counters on a plain 256 MiB copy, averaged over the launches that do work (a
# speculative launch whose device-side predicate is off exits at once; the HIP-event accounting skips it
# too); the summaries are under profiles/.  A figure is valid only for the kernel source it was measured on
# (sha256 of its files, in order).
GEMM_TRAFFIC = {"k_gemm_mfma": {"sources": ["paper_2408_10369_amd/csrc/k_gemm.hip",
                                            "paper_2408_10369_amd/csrc/mfma_tile.h",
                                            "paper_2408_10369_amd/csrc/mfma_tile2.h"],
                                "sha256": "048b481c700004740b8aec997fcf49a28e2108e75bea6ae05bc17f17331ab897",
                                "bytes_per_launch": 451.2e6}}


def measured_traffic(kernel):
    import hashlib
    rec = GEMM_TRAFFIC.get(kernel)
    if rec is None or rec["sha256"] is None:
        return None
    h = hashlib.sha256()
    try:
        for src in rec["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except OSError:
        return None
    return rec["bytes_per_launch"] if h.hexdigest() == rec["sha256"] else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-schedule variant of the main step (its launches then stay out of a trace)")
    ap.add_argument("--cpu-sample-rows", type=int, default=0,
                    help="bound the oracle's closure rows per graph (0: all rows)")
    ap.add_argument("--workloads", default="c1,batch,batch_queries,programs,stream,isforeign,dynamic,samegen,io",
                    help="held-out workloads measured after the main one, plain vs learned schedule (comma list of "
                         "c1, batch, batch_queries, programs, stream, isforeign, dynamic, samegen, io; empty for none)")
    ap.add_argument("--stream-queries", type=int, default=10000,
                    help="queries of the n=65,536 stream to run (a prefix of the 10,000)")
    ap.add_argument("--workloads-only", action="store_true",
                    help="skip the main workload and print only the listed workloads (for profiling them)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB device-to-device copy (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus %d is not supported "
                          "(each query row and graph is independent, see the sharding notes in DESIGN.md)"
                          % args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2408_10369_amd as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": 3}))
        return
    ctx = B.Context(0)
    if args.workloads_only:
        print(json.dumps({"workloads": run_workloads(ctx, args)}), flush=True)
        ctx.close()
        return
    n = 16384
    graphs = []
    for pi in range(len(gen.C2_PROBS)):
        _, s, d = gen.c2(pi)
        qs = []
        for ki in range(len(gen.C2_KS)):
            srcs = gen.c2_sources(pi, ki)
            r, c = gen.query_lists(srcs)
            qs.append((torch.as_tensor(r).to(dev), torch.as_tensor(c).to(dev), len(srcs)))
        graphs.append(dict(p=gen.C2_PROBS[pi], s=torch.as_tensor(s).to(dev), d=torch.as_tensor(d).to(dev),
                           m=len(s), queries=qs,
                           R=ctx.zeros(n, n), Rstar=ctx.zeros(n, n),
                           V=[ctx.zeros(k, n) for (_, _, k) in qs], Vs=[ctx.zeros(k, n) for (_, _, k) in qs]))
    torch.cuda.synchronize()

    # product launches of the timed steps, per kernel (0 VALU, 1 MFMA): RMS squarings and dense selection rounds
    prod = {arm: {"ms": 0.0, "ops": 0, "launches": 0, "issued": 0} for arm in KERNELS}
    # the matrix-core launches of each graph's closure, for the spread of the per-launch rates
    spread = [{"ms": 0.0, "ops": 0, "launches": 0, "issued": 0} for _ in range(len(graphs))]
    smp_rec = {"ms": 0.0, "rows": 0}
    gather_rec = {"ms": 0.0, "bytes": 0, "launches": 0}

    def add_spread(gi, st):
        sp = spread[gi]
        sp["ms"] += st["product_ms_mfma"]
        sp["ops"] += st["product_bool_ops_mfma"]
        sp["launches"] += st["products_mfma"]
        sp["issued"] += st["mfma_ops_issued"]

    def add_products(st):
        mf = prod[1]
        mf["ms"] += st["product_ms_mfma"]
        mf["ops"] += st["product_bool_ops_mfma"]
        mf["launches"] += st["products_mfma"]
        mf["issued"] += st["mfma_ops_issued"]
        va = prod[0]
        va["ms"] += st["product_ms"] - st["product_ms_mfma"]
        va["ops"] += st["product_bool_ops"] - st["product_bool_ops_mfma"]
        va["launches"] += st["products"] - st["products_mfma"]
    per_graph = []

    def step(opts=None):
        # the timed step: the edge lists are packed without a host wait (an out-of-range fact would be
        # latched and reported after the timed region) and no call asks for statistics
        for g in graphs:
            ctx.pack_coo_async(g["s"], g["d"], n, n, out=g["R"])
            ctx.rms(g["R"], n, out=g["Rstar"], opts=opts)
            for qi, (r, c, k) in enumerate(g["queries"]):
                ctx.pack_coo_async(r, c, k, n, out=g["V"][qi])
                ctx.smp(g["R"], n, g["V"][qi], out=g["Vs"][qi], opts=opts)

    def fingerprint():
        torch.cuda.synchronize()
        return [int(_hash_dev(t, W)) for g in graphs for t in [g["Rstar"]] + g["Vs"]]

    def instrumented_step():
        # the same calls with statistics (device times, per-launch product timings, arms), untimed
        for gi, g in enumerate(graphs):
            ctx.pack_coo(g["s"], g["d"], n, n, out=g["R"])
            st = {}
            ctx.rms(g["R"], n, out=g["Rstar"], stats=st)
            smp_ms = []
            for qi, (r, c, k) in enumerate(g["queries"]):
                ctx.pack_coo(r, c, k, n, out=g["V"][qi])
                st2 = {}
                ctx.smp(g["R"], n, g["V"][qi], out=g["Vs"][qi], stats=st2)
                smp_ms.append(st2["device_ms"])
                add_products(st2)
                smp_rec["ms"] += st2["device_ms"]
                smp_rec["rows"] += k
            add_products(st)
            add_spread(gi, st)
            gather_rec["ms"] += st["gather_ms"]
            gather_rec["bytes"] += st["gather_bytes"]
            gather_rec["launches"] += st["gathers"]
            if len(per_graph) < len(graphs):
                per_graph.append({"p": g["p"], "edges": g["m"], "rms_squarings": st["iterations"],
                                  "rms_squarings_by_gather": st["arm_trace"].count(B.ARM_PRODUCT_GATHER),
                                  "rms_ms": round(st["device_ms"], 3), "smp_ms_k1_k64_k1024":
                                  [round(x, 3) for x in smp_ms]})

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.deferred_error()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    # the roofline's launch timings and the per-graph figures come from instrumented steps after the timed
    # region (the same launches, each bracketed by HIP events on its stream)
    isteps = max(1, min(args.steps, 5))
    for _ in range(isteps):
        instrumented_step()
    torch.cuda.synchronize()
    rows_per_step = sum(n + sum(k for (_, _, k) in g["queries"]) for g in graphs)
    value = rows_per_step / (ms_per_step / 1000.0)
    W = torch.randint(-2**62, 2**62, (n * (n // 64),), dtype=torch.int64, device="cuda")
    fp_plain = fingerprint()

    # the same step under the learned schedule (the dispatcher may build a closure by the selection from
    # every source, and picks the selections' arms), timed the same way; its answers must be the plain ones
    learned_opts = B.make_opts(dispatch=B.DISPATCH_LEARNED)
    for _ in range(0 if args.no_learned else args.warmup):
        step(learned_opts)
    torch.cuda.synchronize()
    learned = None
    if not args.no_learned:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(learned_opts)
        torch.cuda.synchronize()
        ms_learned = (time.perf_counter() - t0) * 1000.0 / args.steps
        by_selection = 0
        for g in graphs:
            st = {}
            ctx.rms(g["R"], n, out=g["Rstar"], opts=learned_opts, stats=st)
            by_selection += st["arm"] == B.ARM_SMP_CLOSURE_SELECT
        learned = {"ms_per_step": round(ms_learned, 3), "value": round(rows_per_step / (ms_learned / 1000.0), 1),
                   "speedup_over_plain": round(ms_per_step / ms_learned, 3),
                   "closures_by_selection": by_selection, "closures": len(graphs),
                   "bit_identical": fingerprint() == fp_plain}

    # the dominant kernel: the product kernel with the most device time in the step
    arm = max(prod, key=lambda a: prod[a]["ms"])
    pk = prod[arm]
    avg_launch_ms = pk["ms"] / max(pk["launches"], 1)
    ops_per_launch = pk["ops"] / max(pk["launches"], 1)
    dense_tops = ops_per_launch / (avg_launch_ms / 1000.0) / 1e12 if avg_launch_ms > 0 else 0.0
    kname, kdesc, bound, peak = KERNELS[arm]
    # work done: the matrix-core operations the launches actually issued (saturated output tiles are copied
    # and all-zero words of k skipped, so a launch issues less than the dense count of its product); the
    # VALU kernel issues what it counts
    work_per_launch = (pk["issued"] if arm == 1 else pk["ops"]) / max(pk["launches"], 1)
    achieved = work_per_launch / (avg_launch_ms / 1000.0) / 1e12 if avg_launch_ms > 0 else 0.0
    roofline = {"bound": bound, "kernel": "%s (%s; every launch of it in the step: RMS squarings and dense "
                                          "selection rounds)" % (kname, kdesc),
                "achieved": round(achieved, 2), "peak": round(peak, 1), "unit": "Tbool-op/s",
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(kname),
                "traffic_unit": "HBM bytes per launch",
                # A, B^T, C_old and C of an n x n squaring, n / 8 bytes a row
                "algorithmic_bytes_per_launch": 4 * n * (n // 8),
                "work": "operations issued by the launches (not the dense count of the products)",
                "work_per_launch": round(work_per_launch), "avg_launch_ms": round(avg_launch_ms, 4),
                "launches_per_step": pk["launches"] // isteps,
                "dense_count_rate": round(dense_tops, 2),
                "frac_dense_count": round(dense_tops / peak, 4),
                "issued_fraction_of_dense_count": round(work_per_launch / max(ops_per_launch, 1), 4),
                "other_product_kernel_ms_per_step": round(sum(prod[a]["ms"] for a in prod if a != arm) / isteps,
                                                          3)}
    if arm == 1:
        # the per-graph spread of the launches: average launch time and issued rate of each closure's
        # matrix-core squarings
        roofline["launch_spread"] = [
            {"p": graphs[i]["p"], "launches_per_step": sp["launches"] // isteps,
             "avg_launch_ms": round(sp["ms"] / max(sp["launches"], 1), 4),
             "issued_frac": round(sp["issued"] / (sp["ms"] / 1000.0) / 1e12 / peak, 4) if sp["ms"] > 0 else None,
             "issued_fraction_of_dense_count": round(sp["issued"] / max(sp["ops"], 1), 4)}
            for i, sp in enumerate(spread)]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(graphs, n, args.cpu_sample_rows)

    # the RMS squarings done by row gathers (k_gather_rows_w, with k_gather_rows_q for the queued pieces of
    # heavy rows) against the HBM roofline: per squaring of an R with b set bits, the n rows of R and the b
    # source rows read and the n result rows written, n / 8 bytes each, over the squaring's HIP-event time
    gather_hbm = None
    if gather_rec["launches"] and gather_rec["ms"] > 0:
        gbs = gather_rec["bytes"] / (gather_rec["ms"] / 1e3) / 1e9
        gather_hbm = {"bound": "hbm", "kernel": "k_gather_rows_w + k_gather_rows_q (RMS squarings of a sparse R)",
                      "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                      "launches_per_step": gather_rec["launches"] // isteps,
                      "avg_launch_ms": round(gather_rec["ms"] / gather_rec["launches"], 4),
                      "bytes_per_launch": round(gather_rec["bytes"] / gather_rec["launches"]),
                      "bytes": "per squaring of an R with b set bits: (2n + b) rows of n/8 bytes"}
    # the selections' data movement against the HBM roofline: query rows read and answer rows written
    # (n / 8 bytes each; the edge index and the relation's rows read on the way are not counted)
    smp_bytes = 2 * smp_rec["rows"] * (n // 8)
    smp_hbm = {"bound": "hbm (latency at few rows)", "rows_per_step": smp_rec["rows"] // isteps,
               "device_ms_per_step": round(smp_rec["ms"] / isteps, 3),
               "rows_per_s": round(smp_rec["rows"] / (smp_rec["ms"] / 1e3), 1) if smp_rec["ms"] > 0 else None,
               "achieved_GB_per_s": round(smp_bytes / (smp_rec["ms"] / 1e3) / 1e9, 2) if smp_rec["ms"] > 0 else None,
               "peak_GB_per_s": 8000.0,
               "frac": round(smp_bytes / (smp_rec["ms"] / 1e3) / 8e12, 5) if smp_rec["ms"] > 0 else None,
               "bytes": "query rows read + answer rows written, n/8 bytes each"}
    out = {
        "metric": "closure/SMP queries per sec and Bool-op TOPS vs roofline",
        "value": round(value, 1), "unit": "query rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 bit-packed AND/OR (VALU kernels); e2m1 (fp4) matrix-core products with fp32 accumulation "
                 "and a > 0 threshold (the dominant kernel)",
        "data": "synthetic",
        "config": {"workload": "ER digraph density sweep n=16384, p in {1e-4,5e-4,1e-3,5e-3,1e-2}: "
                               "pack + BMLP-RMS closure + BMLP-SMP from k=1,64,1024 sources per graph",
                   "n": n, "graphs": len(graphs), "query_rows_per_step": rows_per_step},
        "learned": learned,
        "roofline": roofline, "gather_hbm": gather_hbm, "cpu_baseline": cpu, "smp_hbm": smp_hbm,
        "per_graph": per_graph,
    }
    wl = [w for w in args.workloads.split(",") if w]
    if wl:
        # the main workload's buffers are no longer needed
        del graphs
        torch.cuda.empty_cache()
        out["workloads"] = run_workloads(ctx, args)
    print(json.dumps(out), flush=True)
    ctx.close()


def run_workloads(ctx, args):
    res = {}
    for name in [w for w in args.workloads.split(",") if w]:
        fn = {"c1": wl_c1, "batch": wl_batch, "batch_queries": wl_batch_queries, "programs": wl_programs,
              "stream": wl_stream,
              "isforeign": wl_isforeign, "dynamic": wl_dynamic, "samegen": wl_samegen, "io": wl_io}[name]
        res[name] = fn(ctx, args)
        print(json.dumps({"workload_done": name}), file=sys.stderr, flush=True)
    return res


def _modes(B):
    return {"plain": B.make_opts(dispatch=B.DISPATCH_PLAIN), "learned": B.make_opts(dispatch=B.DISPATCH_LEARNED)}


def _hash_dev(t, W):
    """Order-dependent 64-bit fingerprint of a bit matrix (wrapping integer arithmetic), left on the device."""
    flat = t.reshape(-1)
    return (flat * W[: flat.numel()]).sum()


def _hash(t, W):
    return int(_hash_dev(t, W).item())


def wl_batch(ctx, args, with_closure=True):
    """512 uneven graphs (n log-uniform in [64, 4096], mean degree U(2, 8), 64 queries each): every
    closure and every query answer in one hipGraph launch; plain vs learned schedule.  The learned schedule
    asks the dispatcher model on the device, per graph, whether to answer the queries off the closure or by
    per-row selection."""
    import torch

    import gen
    import paper_2408_10369_amd as B

    bg = gen.batch_graphs()
    graphs = []
    for g in bg:
        R = ctx.pack_coo(torch.as_tensor(g.src), torch.as_tensor(g.dst), g.n, g.n)
        r, c = gen.query_lists(g.srcs)
        V = ctx.pack_coo(torch.as_tensor(r), torch.as_tensor(c), len(g.srcs), g.n)
        graphs.append({"n": g.n, "R1": R, "closure": torch.zeros_like(R) if with_closure else None, "V": V,
                       "Vstar": torch.zeros_like(V)})
    W = torch.randint(-2**62, 2**62, (4096 * 64,), dtype=torch.int64, device="cuda")
    res, fp = {}, {}
    modes = _modes(B)
    modes["forced_closure"] = B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE)
    modes["forced_selection"] = B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_SPARSE)
    for mode, o in modes.items():
        ctx.batched(graphs, opts=o)
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            ctx.batched(graphs, opts=o)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        st = {}
        ctx.batched(graphs, opts=o, stats=st)
        fp[mode] = [((_hash(g["closure"], W) if with_closure else 0), _hash(g["Vstar"], W)) for g in graphs]
        ms = sorted(ts)[len(ts) // 2]
        res[mode] = {"ms": round(ms, 3), "graphs_per_s": round(len(graphs) / (ms / 1e3), 1),
                     "bool_ops": st["bool_ops"], "tops": round(st["bool_ops"] / (ms / 1e3) / 1e12, 1),
                     "graphs_answered_off_closure": st["arm_trace"][0],
                     "graphs_answered_by_selection": st["arm_trace"][1]}
    best_static = min(res["forced_closure"]["ms"], res["forced_selection"]["ms"])
    what = "closure + 64 queries each" if with_closure else "64 queries each, closures not requested"
    return {"workload": "512 ER digraphs, n log-uniform [64,4096], mean degree U(2,8), %s, one hipGraph launch" % what,
            "plain": res["plain"], "learned": res["learned"],
            "forced_ms": {"closure": res["forced_closure"]["ms"], "selection": res["forced_selection"]["ms"]},
            "rules": "plain answers each query row by a selection inside the graph (the paper's mapping); learned "
                     "asks the dispatcher model on the device, per graph, between the answers off the closure and "
                     "per-row selection" + ("" if with_closure else ", and squares only the graphs it reads off"),
            "speedup_learned_over_plain": round(res["plain"]["ms"] / res["learned"]["ms"], 3),
            "learned_over_best_static_policy": round(res["learned"]["ms"] / best_static, 3),
            "bit_identical": all(h == fp["plain"] for h in fp.values())}


def wl_batch_queries(ctx, args):
    """The same 512 graphs and queries with no closure requested: answering a graph's queries off its
    closure now costs the closure, so the per-graph choice matters."""
    return wl_batch(ctx, args, with_closure=False)


def wl_programs(ctx, args):
    """100 linear-recursion programs p <- r_base; p <- r_step, p over the synthetic multi-relational
    graph (14,951 entities, 1,345 relations, 592,000 facts); plain vs learned schedule."""
    import torch

    import gen
    import paper_2408_10369_amd as B

    mr = gen.multirel()
    progs = gen.programs(mr, count=100, base_seed=4000)
    n = mr.n
    packed = {}
    for (b, s) in progs:
        for r in (b, s):
            if r not in packed:
                packed[r] = ctx.pack_coo(torch.as_tensor(mr.rel_src[r]), torch.as_tensor(mr.rel_dst[r]), n, n)
    outs = [ctx.zeros(n, n) for _ in progs]  # one output per program (28 MB each), hashed after timing
    W = torch.randint(-2**62, 2**62, (outs[0].numel(),), dtype=torch.int64, device="cuda")
    modes = _modes(B)
    # every call-level arm the learned schedule chooses among, forced on every program: the per-program
    # best of these in hindsight is the reference for the regret of both schedules
    forced = {"cols_adaptive": (B.ARM_COMPOSE_SEMINAIVE, B.ARM_SMP_ADAPTIVE),
              "cols_one_launch": (B.ARM_COMPOSE_SEMINAIVE, B.ARM_SMP_SPARSE),
              "rows": (B.ARM_COMPOSE_ROWWISE, B.ARM_AUTO), "closure": (B.ARM_COMPOSE_RMS, B.ARM_AUTO)}
    for name, (carm, sarm) in forced.items():
        modes["forced_" + name] = B.make_opts(dispatch=B.DISPATCH_FORCED, compose_arm=carm, smp_arm=sarm)
    for i, (b, s) in enumerate(progs[:4]):
        for o in modes.values():
            ctx.compose_linear(packed[b], packed[s], n, out=outs[i], opts=o)
    res, fp, dev_ms = {}, {}, {}
    for mode, o in modes.items():
        arms, per = {}, []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, (b, s) in enumerate(progs):
            st = {}
            ctx.compose_linear(packed[b], packed[s], n, out=outs[i], opts=o, stats=st)
            arms[st["arm"]] = arms.get(st["arm"], 0) + 1
            per.append(st["device_ms"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        fp[mode] = [_hash(P, W) for P in outs]
        dev_ms[mode] = per
        res[mode] = {"ms": round(ms, 2), "device_ms": round(sum(per), 2),
                     "programs_per_s": round(len(progs) / (ms / 1e3), 2),
                     "arms": {str(k): v for k, v in sorted(arms.items())}}
    best = [min(dev_ms["forced_" + f][i] for f in forced) for i in range(len(progs))]

    def regret(mode):
        return round(sum(dev_ms[mode][i] / best[i] for i in range(len(progs))) / len(progs), 3)

    for mode in ("plain", "learned"):
        res[mode]["mean_time_over_best_arm"] = regret(mode)
    return {"workload": "100 programs over 14,951 entities / 1,345 relations / 592,000 facts (held-out seeds)",
            "plain": res["plain"], "learned": res["learned"],
            "forced_ms": {k[7:]: v["ms"] for k, v in res.items() if k.startswith("forced_")},
            "best_arm_in_hindsight_ms": round(sum(best), 2),
            "speedup_learned_over_plain": round(res["plain"]["ms"] / res["learned"]["ms"], 3),
            "bit_identical": all(h == fp["plain"] for h in fp.values())}


def wl_stream(ctx, args):
    """A stream of selection queries (k log-uniform in [1, 4096]) over one scale-free digraph,
    n = 65,536, m = 262,144, answered through a session; plain vs learned schedule.  The timed pass gives
    each query as its k source constants and asks for no statistics (the arm that served a query is read
    on the host); the answers are fingerprinted in a second, untimed pass over the first queries, given
    as bit rows through the general query entry point."""
    import torch

    import gen
    import paper_2408_10369_amd as B

    n = 65536
    s, d = gen.scalefree_digraph()
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    queries = gen.query_stream(count=args.stream_queries)
    qs = [torch.as_tensor(q).cuda() for q in queries]  # each query: its k source constants (int32)
    V = ctx.zeros(4096, n)
    Vs = ctx.zeros(4096, n)
    W = torch.randint(-2**62, 2**62, (Vs.numel(),), dtype=torch.int64, device="cuda")
    res, fp = {}, {}
    modes = _modes(B)
    # the plain schedule answers every query of this stream by the one-launch sparse selection; the other
    # static policies build the closure at the first query (by BMLP-RMS, or by the selection from every
    # source) and read every answer off it
    modes["forced_closure"] = B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE)
    modes["forced_closure_select"] = B.make_opts(dispatch=B.DISPATCH_FORCED, smp_arm=B.ARM_SMP_CLOSURE_SELECT)
    rows_total = sum(len(q) for q in queries)
    nverify = min(len(queries), 500)
    for mode, o in modes.items():
        arms = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        closure_at = None
        with ctx.graph(R, n) as g:
            for qi, src in enumerate(qs):
                g.query_sources(src, Vs[:src.numel()], opts=o)
                a = g.last_arm
                arms[a] = arms.get(a, 0) + 1
                if closure_at is None and a in (B.ARM_SMP_CLOSURE, B.ARM_SMP_CLOSURE_SELECT):
                    closure_at = qi  # the closure is built by the first query it answers
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
        ctx.deferred_error()
        # fingerprints of the answers to the first queries, in a pass of their own
        hs = []
        with ctx.graph(R, n) as g:
            for qi in range(nverify):
                # the same queries as bit rows through the general entry point
                k = len(queries[qi])
                r, c = (torch.as_tensor(x).cuda() for x in gen.query_lists(queries[qi]))
                ctx.pack_coo_async(r, c, k, n, out=V[:k])
                g.query(V[:k], out=Vs[:k], opts=o)
                hs.append(_hash_dev(Vs[:k], W))
        fp[mode] = [int(h) for h in torch.stack(hs).cpu()]
        # bytes a query moves at the least: its rows read, one closure row per source read, its answers
        # written (n / 8 bytes each) -- the rows of a read-off answer
        hbm_bytes = 3 * rows_total * (n // 8)
        res[mode] = {"ms": round(ms, 1), "queries_per_s": round(len(queries) / (ms / 1e3), 1),
                     "rows_per_s": round(rows_total / (ms / 1e3), 1),
                     "arms": {str(k): v for k, v in sorted(arms.items())}, "closure_built_at_query": closure_at,
                     "hbm": {"bytes": hbm_bytes, "achieved_GB_per_s": round(hbm_bytes / (ms / 1e3) / 1e9, 1),
                             "frac": round(hbm_bytes / (ms / 1e3) / 8e12, 4),
                             "floor_ms_at_8TBps": round(hbm_bytes / 8e12 * 1e3, 2)}}
    return {"workload": "scale-free digraph n=65536 m=262144, %d queries, k log-uniform [1,4096] "
                        "(%d rows), one session" % (len(queries), rows_total),
            "plain": res["plain"], "learned": res["learned"], "forced_closure": res["forced_closure"],
            "forced_closure_select": res["forced_closure_select"],
            "arm_codes": {"3": "one-launch selection", "4": "read off the closure (query 0 of forced_closure: "
                          "built by BMLP-RMS)", "13": "the closure built by the selection from every source"},
            "speedup_learned_over_plain": round(res["plain"]["ms"] / res["learned"]["ms"], 3),
            "learned_over_best_static_policy": round(
                res["learned"]["ms"] / min(res[m]["ms"] for m in ("plain", "forced_closure", "forced_closure_select")),
                3),
            "bit_identical": all(h == fp["plain"] for h in fp.values()),
            "bit_identical_checked_queries": nverify}


def wl_c1(ctx, args):
    """The smallest configuration as latency: BMLP-RMS on the n = 1,000, p = 0.002 digraph and BMLP-SMP from
    its 10 sources, one call at a time (median of 50 calls, host wall time around each call)."""
    import torch

    import gen
    import paper_2408_10369_amd as B

    n, s, d, srcs = gen.c1()
    R = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    r, c = gen.query_lists(srcs)
    V = ctx.pack_coo(torch.as_tensor(r), torch.as_tensor(c), len(srcs), n)
    out = {}
    for name, fn in (("rms", lambda: ctx.rms(R, n)), ("smp_10_sources", lambda: ctx.smp(R, n, V))):
        ref = fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(50):
            t0 = time.perf_counter()
            got = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e6)
        st = {}
        (ctx.rms(R, n, stats=st) if name == "rms" else ctx.smp(R, n, V, stats=st))
        out[name] = {"us_median": round(sorted(ts)[25], 1), "us_min": round(min(ts), 1),
                     "device_us": round(st["device_ms"] * 1e3, 1), "iterations": st["iterations"],
                     "bit_identical_across_calls": bool(torch.equal(ref, got))}
    return {"workload": "ER digraph n=1000, p=0.002 (%d edges): closure and 10-source selection latency" % len(s),
            **out}


def wl_isforeign(ctx, args):
    """The stratified program P3 u P4 u P5 (hasPlace = contains+, indirectlyPartOf by linear
    recursion over the inverse of hasPlace, isForeign by negation) on a synthetic geography shaped
    like the FB15K-237 location facts: 14,541 constants, 4,172 contains + 3,811 adjoins facts, every
    constant a location.  One run is the whole program from the fact lists on the device to the
    three relations; plain vs learned schedule, and each composition route forced."""
    import numpy as np
    import torch

    import gen
    import paper_2408_10369_amd as B
    from paper_2408_10369_amd.programs import is_foreign

    g = gen.geo()
    n = g.n
    dev = "cuda:0"
    facts = [torch.as_tensor(a).to(dev) for a in (g.contains_src, g.contains_dst, g.adjoins_src, g.adjoins_dst)]
    loc = torch.arange(n, dtype=torch.int32, device=dev)
    modes = _modes(B)
    forced = {"cols_adaptive": (B.ARM_COMPOSE_SEMINAIVE, B.ARM_SMP_ADAPTIVE),
              "cols_one_launch": (B.ARM_COMPOSE_SEMINAIVE, B.ARM_SMP_SPARSE),
              "rows": (B.ARM_COMPOSE_ROWWISE, B.ARM_AUTO), "closure": (B.ARM_COMPOSE_RMS, B.ARM_AUTO)}
    for name, (carm, sarm) in forced.items():
        modes["forced_" + name] = B.make_opts(dispatch=B.DISPATCH_FORCED, compose_arm=carm, smp_arm=sarm)
    W = torch.randint(-2**62, 2**62, (n * ((n + 63) // 64),), dtype=torch.int64, device=dev)

    def run(o, st=None):
        return is_foreign(ctx, n, (facts[0], facts[1]), (facts[2], facts[3]), loc, opts=o, stats=st)

    res, fp = {}, {}
    for mode, o in modes.items():
        run(o)
        torch.cuda.synchronize()
        ts = []
        for _ in range(7):
            t0 = time.perf_counter()
            out = run(o)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        st = {}
        out = run(o, st)
        fp[mode] = [_hash(t, W) for t in out]
        ms = sorted(ts)[len(ts) // 2]
        res[mode] = {"ms": round(ms, 3), "compose_arm": st.get("arm"), "compose_device_ms": st.get("device_ms")}
    facts_out = {key: int(np.unpackbits(t.cpu().numpy().view(np.uint8)).sum())
                 for key, t in zip(("hasPlace", "indirectlyPartOf", "isForeign"), out)}
    r = {"workload": "P3 u P4 u P5 isForeign, n=14,541 constants, 7,983 facts (4,172 contains, 3,811 adjoins), "
                     "every constant a location; pack + RMS + TRANSP + OR + composition + location product + NEG/AND",
         "plain": res["plain"], "learned": res["learned"],
         "forced_ms": {k[7:]: v["ms"] for k, v in res.items() if k.startswith("forced_")},
         "derived_facts": facts_out,
         "speedup_learned_over_plain": round(res["plain"]["ms"] / res["learned"]["ms"], 3),
         "paper_reported_s": {"value": 2.09, "system": "BMLP-RMS in PyTorch on an A100 (FB15K-237 itself)"},
         "bit_identical": all(h == fp["plain"] for h in fp.values())}
    if not args.no_cpu_baseline:
        r["cpu_baseline"] = cpu_baseline_isforeign(g)
    return r


def wl_dynamic(ctx, args):
    """Closure maintenance under insertions: the closure of the sparsest density-sweep graph
    (n = 16,384, p = 1e-4, 26,879 edges) updated in place with a batch of b new random edges, against
    recomputing the closure of the enlarged relation from scratch; both results must be identical."""
    import numpy as np
    import torch

    import gen

    n, s, d = gen.c2(0)
    dev = "cuda:0"
    R0 = ctx.pack_coo(torch.as_tensor(s), torch.as_tensor(d), n, n)
    T0 = ctx.rms(R0, n)
    W = torch.randint(-2**62, 2**62, (T0.numel(),), dtype=torch.int64, device=dev)
    rng = np.random.default_rng(31337)
    res = {}
    for b in (1, 16, 256, 4096):
        es = torch.as_tensor(rng.integers(0, n, b).astype(np.int32)).to(dev)
        ed = torch.as_tensor(rng.integers(0, n, b).astype(np.int32)).to(dev)
        T = T0.clone()
        ctx.closure_insert(T, n, es, ed)  # warm-up (workspace)
        ts = []
        for _ in range(5):
            T.copy_(T0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.closure_insert(T, n, es, ed)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        inc_ms = sorted(ts)[len(ts) // 2]
        # from scratch: pack the enlarged edge list and take its closure
        us = torch.cat([torch.as_tensor(s).to(dev), es])
        ud = torch.cat([torch.as_tensor(d).to(dev), ed])
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R = ctx.pack_coo(us, ud, n, n)
            Tf = ctx.rms(R, n)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        full_ms = sorted(ts)[len(ts) // 2]
        res[str(b)] = {"insert_ms": round(inc_ms, 3), "recompute_ms": round(full_ms, 3),
                       "speedup": round(full_ms / inc_ms, 1), "bit_identical": _hash(T, W) == _hash(Tf, W)}
    return {"workload": "closure of the n=16,384 p=1e-4 sweep graph, batches of b random edge insertions "
                        "(in place) vs the closure recomputed from the enlarged edge list",
            "by_batch": res, "bit_identical": all(v["bit_identical"] for v in res.values())}


def wl_samegen(ctx, args):
    """Same-generation, p <- flat; p <- up, p, down, on a random forest of n = 16,384 nodes (8 trees,
    up to 4 children per node): the two-sided linear recursion with the library's choice per round
    (row gathers while an operand is sparse) against every product on the bit-packed VALU kernel and
    on the matrix cores."""
    import numpy as np
    import torch

    import gen
    import paper_2408_10369_amd as B

    f = gen.forest()
    n = f.n
    roots = np.unique(f.root).astype(np.int32)

    def pk(s, d):
        return ctx.pack_coo(torch.as_tensor(np.asarray(s, np.int32)), torch.as_tensor(np.asarray(d, np.int32)), n, n)

    flat, up, down = pk(roots, roots), pk(f.child, f.parent), pk(f.parent, f.child)
    out = ctx.zeros(n, n)
    W = torch.randint(-2**62, 2**62, (out.numel(),), dtype=torch.int64, device="cuda")
    modes = {"auto": None,
             "valu_products": B.make_opts(dispatch=B.DISPATCH_FORCED, product_arm=B.ARM_PRODUCT_VALU),
             "mfma_products": B.make_opts(dispatch=B.DISPATCH_FORCED, product_arm=B.ARM_PRODUCT_MFMA)}
    res, fp = {}, {}
    for name, o in modes.items():
        ctx.compose_two_sided(flat, up, down, n, out=out, opts=o)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = {}
            ctx.compose_two_sided(flat, up, down, n, out=out, opts=o, stats=st)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        fp[name] = _hash(out, W)
        res[name] = {"ms": round(sorted(ts)[1], 3), "rounds": st["iterations"]}
    facts = int(np.unpackbits(out.cpu().numpy().view(np.uint8)).sum())
    return {"workload": "same-generation on a random forest, n=16,384 nodes, 8 trees, depth %d" % int(f.depth.max()),
            "by_mode": res, "derived_facts": facts, "bit_identical": len(set(fp.values())) == 1}


def wl_io(ctx, args):
    """Facts in and out at device speed: packing the densest sweep graph's 2,686,179 edge pairs into an
    n = 16,384 bit matrix, and decoding the isForeign relation of the knowledge-graph program (211 M
    facts) into sorted (row, column) int32 pairs."""
    import numpy as np
    import torch

    import gen
    from paper_2408_10369_amd.programs import is_foreign

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return sorted(ts)[len(ts) // 2]

    n, s, d = gen.c2(4)
    S, D = torch.as_tensor(s).cuda(), torch.as_tensor(d).cuda()
    R = ctx.zeros(n, n)
    pack_ms = timed(lambda: ctx.pack_coo(S, D, n, n, out=R))
    g = gen.geo()
    facts = [torch.as_tensor(a).cuda() for a in (g.contains_src, g.contains_dst, g.adjoins_src, g.adjoins_dst)]
    loc = torch.arange(g.n, dtype=torch.int32, device="cuda")
    _, _, foreign = is_foreign(ctx, g.n, (facts[0], facts[1]), (facts[2], facts[3]), loc)
    out = {}
    unpack_ms = timed(lambda: out.__setitem__("rc", ctx.unpack_coo(foreign, g.n)), reps=3)
    m = int(out["rc"][0].numel())
    return {"workload": "pack 2,686,179 edges into a 16,384 x 16,384 bit matrix; decode the 14,541 x 14,541 "
                        "isForeign relation into sorted int32 (row, column) pairs",
            "pack": {"ms": round(pack_ms, 3), "facts": len(s), "facts_per_s": round(len(s) / (pack_ms / 1e3), 1)},
            "unpack": {"ms": round(unpack_ms, 3), "facts": m, "facts_per_s": round(m / (unpack_ms / 1e3), 1),
                       "output_GB_per_s": round(8 * m / (unpack_ms / 1e3) / 1e9, 1)}}


def cpu_baseline_isforeign(g):
    """The oracle's bit-row pipeline for the same program on the same facts (whole program)."""
    import oracle

    oracle.is_foreign_rows(g.n, (g.contains_src, g.contains_dst), (g.adjoins_src, g.adjoins_dst))
    t0 = time.perf_counter()
    oracle.is_foreign_rows(g.n, (g.contains_src, g.contains_dst), (g.adjoins_src, g.adjoins_dst))
    ms = (time.perf_counter() - t0) * 1e3
    return {"ms": round(ms, 1), "cores": oracle.last_threads, "kind": "oracle",
            "sample": "the whole program once: closure rows by BFS, composition rows by BFS, numpy NEG/AND"}


def cpu_baseline(graphs, n, sample_rows):
    """The oracle (per-source BFS) on the same workload as one step: every
    closure row of every graph and every SMP query row.  ``sample_rows`` > 0
    bounds the closure part to that many random rows per graph instead."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(12345)
    t_total = 0.0
    rows_total = 0
    threads = 0
    # the oracle's rows are compared with the last timed step's outputs (closures and answers), bit for bit
    compared, mismatched = 0, 0
    for g in graphs:
        s = g["s"].cpu().numpy()
        d = g["d"].cpu().numpy()
        rows = None if sample_rows <= 0 else np.sort(rng.choice(n, sample_rows, replace=False))
        t0 = time.perf_counter()
        want = oracle.closure_rows(n, s, d, rows=rows)
        t_total += time.perf_counter() - t0
        rows_total += n if rows is None else len(rows)
        threads = oracle.last_threads
        got = g["Rstar"].cpu().numpy().view(np.uint64)
        got = got if rows is None else got[rows]
        compared += want.shape[0]
        mismatched += int((got != want).any(axis=1).sum())
        for V, Vs in zip(g["V"], g["Vs"]):
            Vh = V.cpu().numpy().view(np.uint64)
            t0 = time.perf_counter()
            want = oracle.smp(n, s, d, Vh)
            t_total += time.perf_counter() - t0
            rows_total += Vh.shape[0]
            compared += want.shape[0]
            mismatched += int((Vs.cpu().numpy().view(np.uint64) != want).any(axis=1).sum())
    # the same oracle on one thread, on 64 random closure rows per graph
    t1, rows1 = 0.0, 0
    for g in graphs:
        s = g["s"].cpu().numpy()
        d = g["d"].cpu().numpy()
        rows = np.sort(rng.choice(n, 64, replace=False))
        t0 = time.perf_counter()
        oracle.closure_rows(n, s, d, rows=rows, threads=1)
        t1 += time.perf_counter() - t0
        rows1 += len(rows)
    what = "all closure rows" if sample_rows <= 0 else "%d random closure rows" % sample_rows
    return {"value": round(rows_total / t_total, 1), "unit": "query rows/s", "cores": threads, "kind": "oracle",
            "sample": "%s of each of the %d graphs plus every SMP query row (k=1,64,1024), per-source BFS; "
                      "%d rows in %.2f s" % (what, len(graphs), rows_total, t_total),
            "oracle_parity": {"rows_compared": compared, "rows_differing": mismatched,
                              "bit_exact": mismatched == 0},
            "value_1_thread": round(rows1 / t1, 1),
            "sample_1_thread": "64 random closure rows of each graph on one thread; %d rows in %.2f s" % (rows1, t1)}


if __name__ == "__main__":
    main()
