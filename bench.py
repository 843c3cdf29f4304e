"""Benchmark of the BMLP hot path on one MI355X.

Workload (one "step"): the n = 16,384 directed Erdos-Renyi density sweep,
p in {1e-4, 5e-4, 1e-3, 5e-3, 1e-2} (seeded synthetic graphs shaped like the
paper's DG / DG+partial benchmarks).  For each of the five graphs a step
  1. packs the device-resident COO edge list into the n x n bit matrix,
  2. computes the full closure R1+ with BMLP-RMS (all n groundings r2(X, Y)),
  3. answers SMP queries r2(c, Y) from 1, 64 and 1,024 sources.
Inputs are resident in HBM before the timed region.  The value is answered
query rows per second (a closure answers n rows; an SMP batch answers k).

Also reported: the live roofline of the dominant kernel (the bit-packed
product), measured with HIP events around each product launch on the stream
it runs on, and the CPU oracle timed on a bounded sample of the same
workload on this host's cores.
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

VALU_PEAK_TOPS = 256 * 64 * 2.4e9 * 32 * 2 / 1e12  # bool-ops/s: 64 lanes x 32 bits x (AND+OR) per CU-clock

# HBM bytes per launch of the product kernel on this workload: rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch) scaled by the same counters on a plain 256 MiB copy (fetch x2.000, write x1.000); the summary is
# profiles/k_gemm_valu_er16384_density_sweep.md.  Valid only for the kernel source it was measured on.
GEMM_TRAFFIC = {"source": "paper_2408_10369_amd/csrc/k_gemm.hip",
                "sha256": "5ccb7508fd01657d6439160d53dea3f119adddd9bf423655e162c26ec0ba5de9",
                "bytes_per_launch": 496.6e6}


def measured_traffic():
    import hashlib
    path = os.path.join(ROOT, GEMM_TRAFFIC["source"])
    try:
        digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    except OSError:
        return None
    return GEMM_TRAFFIC["bytes_per_launch"] if digest == GEMM_TRAFFIC["sha256"] else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=0,
                    help="bound the oracle's closure rows per graph (0: all rows)")
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

    prod = {"ms": 0.0, "ops": 0, "launches": 0}
    per_graph = []

    def step(record: bool):
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
            if record:
                prod["ms"] += st["product_ms"]
                prod["ops"] += st["product_bool_ops"]
                prod["launches"] += st["products"]
                if len(per_graph) < len(graphs):
                    per_graph.append({"p": g["p"], "edges": g["m"], "rms_products": st["products"],
                                      "rms_ms": round(st["device_ms"], 3), "smp_ms_k1_k64_k1024":
                                      [round(x, 3) for x in smp_ms]})

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    rows_per_step = sum(n + sum(k for (_, _, k) in g["queries"]) for g in graphs)
    value = rows_per_step / (ms_per_step / 1000.0)

    avg_launch_ms = prod["ms"] / max(prod["launches"], 1)
    ops_per_launch = prod["ops"] / max(prod["launches"], 1)
    achieved_tops = ops_per_launch / (avg_launch_ms / 1000.0) / 1e12 if avg_launch_ms > 0 else 0.0
    roofline = {"bound": "alu", "kernel": "k_gemm_valu (bit-packed Boolean product, RMS squarings)",
                "achieved": round(achieved_tops, 2), "peak": round(VALU_PEAK_TOPS, 1), "unit": "Tbool-op/s",
                "frac": round(achieved_tops / VALU_PEAK_TOPS, 4), "traffic": measured_traffic(),
                "traffic_unit": "HBM bytes per launch",
                "avg_launch_ms": round(avg_launch_ms, 4), "launches_per_step": prod["launches"] // args.steps}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(graphs, n, args.cpu_sample_rows)

    out = {
        "metric": "closure/SMP queries per sec and Bool-op TOPS vs roofline",
        "value": round(value, 1), "unit": "query rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64 bit-packed (AND/OR)", "data": "synthetic",
        "config": {"workload": "ER digraph density sweep n=16384, p in {1e-4,5e-4,1e-3,5e-3,1e-2}: "
                               "pack + BMLP-RMS closure + BMLP-SMP from k=1,64,1024 sources per graph",
                   "n": n, "graphs": len(graphs), "query_rows_per_step": rows_per_step},
        "roofline": roofline, "cpu_baseline": cpu, "per_graph": per_graph,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


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
    for g in graphs:
        s = g["s"].cpu().numpy()
        d = g["d"].cpu().numpy()
        rows = None if sample_rows <= 0 else np.sort(rng.choice(n, sample_rows, replace=False))
        t0 = time.perf_counter()
        oracle.closure_rows(n, s, d, rows=rows)
        t_total += time.perf_counter() - t0
        rows_total += n if rows is None else len(rows)
        threads = oracle.last_threads
        for V in g["V"]:
            Vh = V.cpu().numpy().view(np.uint64)
            t0 = time.perf_counter()
            oracle.smp(n, s, d, Vh)
            t_total += time.perf_counter() - t0
            rows_total += Vh.shape[0]
    what = "all closure rows" if sample_rows <= 0 else "%d random closure rows" % sample_rows
    return {"value": round(rows_total / t_total, 1), "unit": "query rows/s", "cores": threads, "kind": "oracle",
            "sample": "%s of each of the %d graphs plus every SMP query row (k=1,64,1024), per-source BFS; "
                      "%d rows in %.2f s" % (what, len(graphs), rows_total, t_total)}


if __name__ == "__main__":
    main()
