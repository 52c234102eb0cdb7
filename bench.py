"""Benchmark: barrier-filtered contact evaluation on one MI355X.

One step = build_candidates -> filter_pairs -> eval_barrier ->
assemble_grad_hess over the woven yarn patch (32 warp x 32 weft rods, 512
vertices per rod, graded 20-300 um segments, h = 300 um, dhat = 30 um) with
the positions already resident in device memory.  The throughput numerator
is N_c, the number of pairs closer than h (the pairs the path evaluates for
distance and filter); N_act (active pairs) is reported beside it.

Prints one JSON line (see the fields below).  --gpus above 1 is refused: the
path runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic FP64 flops of one active pair by distance kind (PP, PE, PT, EE):
# chain rule through d (about 0.1k / 0.5k / 1.2k / 1.2k), a symmetric
# eigensystem of the translation-free Hessian (n = 0 closed form, 6, 9, 9;
# 4n^3/3 tridiagonalisation + 6n^3 QL with vectors + n^3 reconstruction) and
# the map back to 12 DOFs (0.4k / 0.7k).
FLOPS_PER_KIND = {0: 150.0, 1: 2700.0, 2: 8000.0, 3: 8000.0}
# Algorithmic bytes of one active pair in eval_barrier: pair ids, type, code,
# flags (11 B), four FP64 vertices (96 B), and E, G[12], H[12 x 12] (1256 B).
EVAL_BYTES_PER_PAIR = 11 + 96 + 8 + 96 + 1152
KIND_OF_CODE = np.array([0, 0, 0, 1, 1, 1, 2, 0, 0, 0, 0, 1, 1, 1, 1, 3])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="woven_patch", choices=["woven_patch", "folded_cloth", "helix_loop_rod"])
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--graph", type=int, default=1, help="replay the step as a captured HIP graph")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(sc, n_c_gpu):
    """The oracle, as it stands, on the same workload (swept enumeration,
    derivatives of every active pair); repeated until ~10 s of CPU work."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    reps, t_total, n_c = 0, 0.0, 0
    while t_total < 10.0 and reps < 20:
        t0 = time.perf_counter()
        res = oracle.evaluate(sc, mode=1, derivs=True, nthreads=threads)
        t_total += time.perf_counter() - t0
        n_c = oracle.counts(res)["n_c"]
        reps += 1
    assert n_c == n_c_gpu, (n_c, n_c_gpu)
    return {"value": n_c * reps / t_total, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"whole workload, {reps} evaluation(s) of all pairs with d < h "
                      f"(swept enumeration, FP64, derivatives and projection of every active pair)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2510_10256_amd as bfc

    sc = synth.workload(args.workload)
    prec = bfc.BF_FP64 if args.prec == "fp64" else bfc.BF_MIXED
    dev = torch.device("cuda:0")
    x = torch.tensor(sc.x, dtype=torch.float64, device=dev)
    cs = bfc.ContactScene(sc, prec=prec, device=dev)
    t0 = time.perf_counter()
    cs.run(x)  # sizes the buffers (grows them on overflow, then steps again)
    counts = cs.counts()
    n_c, n_act = counts["n_c"], counts["n_act"]
    codes = cs.a_code[:n_act].cpu().numpy()
    kinds = KIND_OF_CODE[codes]

    stream = torch.cuda.current_stream(dev)
    graph = None
    if args.graph:
        # one step captured as a graph (every launch is on the current stream,
        # no host synchronisation and no allocation inside the step)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            cs.step(x)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            cs.step(x)
        torch.cuda.synchronize()

    def one_step():
        if graph is not None:
            graph.replay()
        else:
            cs.step(x)

    if args.copy_mib > 0:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE counters convert
        # the counters of the path's kernels to bytes
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    st = cs.status(clear=True)
    assert not (st & (bfc.BF_S_CAND_OVERFLOW | bfc.BF_S_ACT_OVERFLOW | bfc.BF_S_BSR_OVERFLOW)), st
    assert cs.counts() == counts, (cs.counts(), counts)

    # timed region: K whole steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        one_step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    ms_per_step = wall * 1e3 / args.steps

    # per-call durations on the launching stream (eager, after the timed region)
    calls = ["build_candidates", "filter_pairs", "eval_barrier", "assemble_grad_hess"]
    fns = [lambda: cs.build_candidates(x), lambda: cs.filter_pairs(x), lambda: cs.eval_barrier(x),
           lambda: cs.assemble_grad_hess()]
    per = {c: [] for c in calls}
    for _ in range(max(10, args.steps // 5)):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record(stream)
        for q, f in enumerate(fns):
            f()
            e[q + 1].record(stream)
        torch.cuda.synchronize()
        for q, c in enumerate(calls):
            per[c].append(e[q].elapsed_time(e[q + 1]))
    call_ms = {c: float(np.mean(v)) for c, v in per.items()}

    # roofline of the per-pair evaluation kernel (the one kernel of eval_barrier)
    eval_ms = call_ms["eval_barrier"]
    flops = float(sum(FLOPS_PER_KIND[int(k)] * int(np.sum(kinds == k)) for k in range(4)))
    bytes_ = float(EVAL_BYTES_PER_PAIR * n_act)
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
    t_fp = flops / (FP64_PEAK_TFLOPS * 1e12)
    if t_hbm >= t_fp:
        roof = {"kernel": "k_eval (eval_barrier)", "bound": "hbm", "achieved": bytes_ / (eval_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"kernel": "k_eval (eval_barrier)", "bound": "alu", "achieved": flops / (eval_ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["units"] = {"active_pairs": n_act, "bytes": bytes_, "fp64_flops": flops,
                     "pairs_by_kind": {k: int(np.sum(kinds == q)) for q, k in enumerate(["PP", "PE", "PT", "EE"])}}

    out = {
        "metric": "filtered contact pairs evaluated/s (dist+filter+grad+Hessian); p50/p99 latency",
        "value": n_c / (ms_per_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": f"{sc.name}: " + ("32 warp x 32 weft rods, 512 vertices per rod, segments "
                                                 "20-300 um, h = 300 um, dhat = 30 um"
                                                 if sc.name == "woven_patch" else sc.name),
                   "n_verts": sc.n_verts, "n_edges": sc.n_edges, "n_tris": sc.n_tris,
                   "N_bp": counts["n_bp"], "N_c": n_c, "N_filt": counts["n_filt"], "N_act": n_act,
                   "nnzb": counts["nnzb"], "graph": bool(args.graph), "precision": args.prec},
        "active_pairs_per_s": n_act / (ms_per_step * 1e-3),
        "call_ms": call_ms,
        "setup_s": time.perf_counter() - t0 - wall,
        "roofline": roof,
    }
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, n_c)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
