"""Benchmark: barrier-filtered contact evaluation on one MI355X.

One step = build_candidates -> filter_pairs -> eval_barrier ->
assemble_grad_hess over the thick shell cloth (256 x 256 vertices, 130,050
triangles, three Z-folds bringing layers within 2 mm, h = 1 mm, dhat =
0.1 mm), the largest single-scene workload, with the positions already
resident in device memory.  The throughput numerator is N_c, the number of
pairs closer than h (the pairs the path evaluates for distance and filter);
N_act (active pairs) is reported beside it.

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
# Algorithmic work per unit of each stage of the step (the path's scope
# table, measurement row): bytes that must cross HBM, and FP64 operations.
#   a1 broad phase: positions and topology in (24 V + 8 E + 12 F), one
#      counting sort of the stored primitives (2 x (8 + 4) B each), the
#      candidate list out (9 B per candidate: i, j, type)
#   a2 narrow phase and filter: 9 B of ids per candidate in, 32 B per active
#      pair out; about 150 FP64 operations per candidate (distance and tests)
#   a3 + a4 evaluation and projection: 8 + 96 + 78 w = 728 B out per active
#      pair (E, G[12], the upper triangle of H in entries of w = 8 B; 416 B
#      in the mixed mode, whose records are FP32: w = 4 B), 11 B of ids in;
#      FP64 operations by kind
#   a5 assembly: 96 + 90 w = 816 B read per active pair (gradient, the ten
#      3 x 3 blocks of the pair's upper triangle; 456 B in the mixed mode),
#      72 B written per block of the matrix and 24 B per vertex (gradient)
A1_BYTES_PER_STORED = 2 * (8 + 4)
CAND_BYTES = 9
A2_FLOPS_PER_CAND = 150.0
A2_BYTES_PER_ACTIVE = 32


def h_entry_bytes(prec):
    """Bytes of one entry of a pair's Hessian record: FP32 in the mixed mode."""
    return 4 if prec == "mixed" else 8


def a3_bytes_per_active(prec):
    return 8 + 96 + 78 * h_entry_bytes(prec) + 11


def a5_bytes_per_active(prec):
    return 96 + 90 * h_entry_bytes(prec)


KIND_OF_CODE = np.array([0, 0, 0, 1, 1, 1, 2, 0, 0, 0, 0, 1, 1, 1, 1, 3])


def friction_bytes_per_pair(prec):
    """Algorithmic bytes of one lagged pair in friction_eval: pair ids and
    type (9 B), lambda, weights[4], normal[3] (64 B), four vertices at x and at
    the lagged positions (192 B), and E, G[12] and the packed upper triangle
    of H[12 x 12] (78 entries) out."""
    return 9 + 64 + 192 + 8 + 96 + 78 * h_entry_bytes(prec)

# HBM bytes per launch of a stage's kernels, counted with rocprofv3 --pmc
# (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
# plain device copy of known size) on the kernel source whose fingerprint is
# given; reported as null once that source changes.
TRAFFIC = {("asm_values", "folded_cloth", None): ("5293752ea332d4d2", 4081.3e6),
           ("asm_values", "folded_cloth", "fp64"): ("5293752ea332d4d2", 4081.3e6),
           ("asm_values", "folded_cloth", "mixed"): ("5293752ea332d4d2", 2887.6e6)}
# the same for the friction kernel (lag at x - 0.02 p; the bytes do not depend on mu), FP64
FRICTION_TRAFFIC_SOURCE = "3adca896ab118311"
FRICTION_TRAFFIC_BYTES = {"woven_patch": 25.4e6, "folded_cloth": 1752.4e6}


def _source_fingerprint(first_line, kernel, headers):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2510_10256_amd", "csrc")
    src = open(os.path.join(csrc, "bfc_kernels.hip")).read()
    a = src.index(first_line)
    b = src.index("\n}\n", src.index(kernel, a)) + 3
    text = "".join(open(os.path.join(csrc, f)).read() for f in headers) + src[a:b]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


# source of the stages whose HBM bytes were counted: sections of
# bfc_kernels.hip (from a first line to the end of a last function) and the
# headers they use
STAGE_SECTIONS = {"asm_values": ([("// Packed pair Hessian:", "__constant__ PkTables kPk"),
                                  ("// Assembly (owner computes)", "void k_row_b_big(")], ("bfc_internal.h",))}


def stage_source_fingerprint(stage):
    """Fingerprint of a stage's kernels' source sections and the headers they use."""
    import hashlib
    sections, headers = STAGE_SECTIONS[stage]
    csrc = os.path.join(ROOT, "paper_2510_10256_amd", "csrc")
    src = open(os.path.join(csrc, "bfc_kernels.hip")).read()
    text = "".join(open(os.path.join(csrc, f)).read() for f in headers)
    for first, last in sections:
        a = src.index(first)
        b = src.index("\n", src.index(last, a))
        if last.startswith("void"):
            b = src.index("\n}\n", src.index(last, a)) + 3
        text += src[a:b]
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def friction_source_fingerprint():
    return _source_fingerprint("// Friction of every active pair at x against the lagged xl",
                               "void k_friction_eval(", ("bfc_geom.h",))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="folded_cloth",
                    choices=["woven_patch", "folded_cloth", "helix_loop_rod", "batch64", "serve256"])
    ap.add_argument("--prec", default=None, choices=["fp64", "mixed"],
                    help="default: fp64 for one scene, mixed for the batch")
    ap.add_argument("--lanes", type=int, default=0, help="batch: concurrent streams in the graph (0 = four)")
    ap.add_argument("--tune", type=int, default=1, help="tune threads per broad-phase query (per scene)")
    ap.add_argument("--budget-gib", type=float, default=None,
                    help="serve: HBM budget; the library's loop counts resident scenes and running steps (default "
                         "4), the Python loop resident scenes with their buffers (default 2)")
    ap.add_argument("--slots", type=int, default=4, help="serve: requests on the device at once")
    ap.add_argument("--requests", type=int, default=300, help="serve: requests per open-loop run")
    ap.add_argument("--native-serve", type=int, default=1,
                    help="serve: 1 runs the requests through the library's serving loop (bf_serve_*); 0 through "
                         "the Python loop over the four calls")
    ap.add_argument("--graph", type=int, default=-1,
                    help="1: replay the step as a captured HIP graph; 0: eager launches (the assembly's structure "
                         "then overlaps the evaluation on a second stream); -1: time both, report the faster")
    ap.add_argument("--path", default="step", choices=["step", "linesearch", "locking"],
                    help="step: the four calls of a Newton step (default); linesearch: swept broad phase, additive "
                         "CCD with the filtered offsets and the energy at the step found (one pass per step); "
                         "locking: contact state at rest of a straight rod and a flat sheet over resolutions, with "
                         "the paper's filter, no filter and culling (the comparison of Fig. self_pushing_toy_example)")
    ap.add_argument("--core-squeeze", type=float, default=0.0,
                    help="step path: scale z by this factor (e.g. 0.88 puts the woven crossings inside the core) and "
                         "mark the pairs inside the core for the temporary zero offset before timing (Sec. 3.4)")
    ap.add_argument("--friction-mu", type=float, default=0.0,
                    help="step path: with mu > 0 the step also evaluates and assembles IPC's lagged friction of the "
                         "active pairs (App. A), lagged at x - 0.02 p (the previous positions; slips of about eps_vh)")
    ap.add_argument("--eps-vh", type=float, default=1.0, help="friction smoothing width in um (sliding speed x dt)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(sc, n_c_gpu, x=None, core=None, friction=None):
    """The oracle, as it stands, on the same workload (swept enumeration,
    derivatives of every active pair, and the lagged friction if given);
    repeated until ~10 s of CPU work."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    reps, t_total, n_c = 0, 0.0, 0
    if friction is not None:
        lag, xlag, mu, eh = friction
    while t_total < 10.0 and reps < 20:
        t0 = time.perf_counter()
        res = oracle.evaluate(sc, x, mode=1, derivs=True, nthreads=threads, core=core)
        if friction is not None:
            oracle.friction_eval(lag, sc.x if x is None else x, xlag, mu, eh, nthreads=threads)
        t_total += time.perf_counter() - t0
        n_c = oracle.counts(res)["n_c"]
        reps += 1
    assert n_c == n_c_gpu, (n_c, n_c_gpu)
    return {"value": n_c * reps / t_total, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"whole workload, {reps} evaluation(s) of all pairs with d < h "
                      f"(swept enumeration, FP64, derivatives and projection of every active pair"
                      + (", lagged friction of every lagged pair" if friction is not None else "") + ")"}, res


def eval_roofline(ms, n_act, kinds, label, prec):
    """Roofline of the per-pair evaluation kernel from its measured time."""
    flops = float(sum(FLOPS_PER_KIND[int(k)] * int(np.sum(kinds == k)) for k in range(4)))
    bytes_ = float(a3_bytes_per_active(prec) * n_act)
    t_hbm = bytes_ / (HBM_PEAK_GBS * 1e9)
    t_fp = flops / (FP64_PEAK_TFLOPS * 1e12)
    if t_hbm >= t_fp:
        roof = {"kernel": label, "bound": "hbm", "achieved": bytes_ / (ms * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"kernel": label, "bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["units"] = {"active_pairs": int(n_act), "bytes": bytes_, "fp64_flops": flops,
                     "pairs_by_kind": {k: int(np.sum(kinds == q)) for q, k in enumerate(["PP", "PE", "PT", "EE"])}}
    return roof


# the stages of one step, the kernels in each, and the row of the path's
# scope table whose work they do
STAGES = [
    ("broad", "a1 broad phase", ["k_bounds", "k_count", "k_scan", "k_scatter", "k_cell_order", "k_pair_count",
                                 "k_pair_emit"]),
    ("narrow", "a2 narrow phase + filter", ["k_narrow"]),
    ("compact", "a2 compaction", ["k_scan", "k_compact", "k_band", "k_exact", "k_dfr_count", "k_exact_emit"]),
    ("eval", "a3 + a4 barrier, derivatives, PSD projection", ["k_eval"]),
    ("asm_structure", "a5 assembly (structure)", ["k_inc_count", "k_scan", "k_inc_fill", "k_row_a", "k_row_a_big"]),
    ("asm_values", "a5 assembly (values)", ["k_scan", "k_row_b", "k_row_b_big"]),
]


def step_roofline(sc, counts, kinds, stage_ms, ms_step, prec):
    """Roofline of the step from the algorithmic work of each stage:
    T_roof = sum over stages of max(bytes / HBM peak, FP64 ops / FP64 peak),
    and the fraction T_roof / T_step; per stage, the same against its
    measured duration.  'dominant' is the longest stage with algorithmic work."""
    V, E, F = sc.n_verts, sc.n_edges, sc.n_tris
    n_bp, n_act, nnzb = counts["n_bp"], counts["n_act"], counts["nnzb"]
    f_eval = float(sum(FLOPS_PER_KIND[int(k)] * int(np.sum(kinds == k)) for k in range(4)))
    work = {  # stage: (bytes, fp64 ops)
        "broad": (24.0 * V + 8.0 * E + 12.0 * F + A1_BYTES_PER_STORED * (E + F) + CAND_BYTES * n_bp, 0.0),
        "narrow": (float(CAND_BYTES * n_bp + A2_BYTES_PER_ACTIVE * n_act), A2_FLOPS_PER_CAND * n_bp),
        "compact": (0.0, 0.0),
        "eval": (float(a3_bytes_per_active(prec) * n_act), f_eval),
        "asm_structure": (0.0, 0.0),
        "asm_values": (float(a5_bytes_per_active(prec) * n_act + 72 * nnzb + 24 * V), 0.0),
    }
    stages = {}
    t_roof = 0.0
    for name, row, kernels in STAGES:
        b, f = work[name]
        t_b, t_f = b / (HBM_PEAK_GBS * 1e9), f / (FP64_PEAK_TFLOPS * 1e12)
        t = max(t_b, t_f)
        t_roof += t
        ms = stage_ms.get(name, -1.0)
        st = {"row": row, "kernels": kernels, "bytes": b, "fp64_flops": f,
              "bound": "hbm" if t_b >= t_f else "fp64", "t_roof_ms": t * 1e3, "measured_ms": ms}
        if ms > 0 and t > 0:
            st["frac"] = t * 1e3 / ms
        stages[name] = st
    # the longest stage with algorithmic work (compaction and the assembly
    # structure move no bytes of their own in the scope table's accounting)
    dom = max((k for k in stages if stages[k]["t_roof_ms"] > 0.0), key=lambda k: stages[k]["measured_ms"])
    d = stages[dom]
    ms = d["measured_ms"]
    if d["bound"] == "hbm":
        dominant = {"kernel": " + ".join(d["kernels"]) + f" ({dom})", "stage": dom, "kernels": d["kernels"],
                    "bound": "hbm", "achieved": d["bytes"] / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s"}
    else:
        dominant = {"kernel": " + ".join(d["kernels"]) + f" ({dom})", "stage": dom, "kernels": d["kernels"],
                    "bound": "fp64", "achieved": d["fp64_flops"] / (ms * 1e-3) / 1e12,
                    "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    dominant["frac"] = dominant["achieved"] / dominant["peak"]
    dominant["kernel_ms"] = ms
    dominant["traffic"] = None
    dominant["units"] = {"candidates": int(n_bp), "active_pairs": int(n_act), "blocks": int(nnzb),
                         "bytes": d["bytes"], "fp64_flops": d["fp64_flops"]}
    return {"t_roof_ms": t_roof * 1e3, "t_step_ms": ms_step, "frac": t_roof * 1e3 / ms_step,
            "stages": stages, "dominant": dominant}


def oracle_errors(g, o, nv, kappa, tau):
    """Errors of the GPU's results against the oracle's on the whole workload:
    the active set and counts (exact), and the worst per-pair and assembled
    errors as fractions of the tolerance (per pair p with band width
    w = a - eta and b_ref = kappa (w/2)^2 ln 2: |dE| <= tau (|E| + b_ref),
    |dG| <= tau (|G| + b_ref/w), |dH+|_F <= tau (|H+|_F + b_ref/w^2); the
    assembled gradient and blocks against the sums of those bounds)."""
    import oracle
    rep = {"tau": tau}
    oc = oracle.counts(o)
    rep["counts_equal"] = all(g["counts"][k] == oc[k] for k in oc)
    act = np.nonzero((o["flags"] & oracle.F_ACTIVE) != 0)[0]
    oi = act[np.lexsort((o["j"][act], o["i"][act], o["ptype"][act]))]
    gi = np.lexsort((g["j"], g["i"], g["ptype"]))
    same = len(gi) == len(oi) and all(np.array_equal(g[k][gi], o[k][oi]) for k in ("ptype", "i", "j"))
    same = same and np.array_equal(g["flags"][gi] & 5, o["flags"][oi] & 5)
    rep["active_set_equal"] = bool(same)
    if not same:
        return rep
    rep["subcase_equal"] = float(np.mean(g["code"][gi] == o["code"][oi])) if len(gi) else 1.0
    feas = (o["flags"][oi] & oracle.F_INFEASIBLE) == 0
    w = (o["a"][oi] - o["eta"][oi])[feas]
    bref = kappa * (w / 2) ** 2 * math.log(2)
    gE, oE = g["E"][gi][feas], o["E"][oi][feas]
    rep["E_pair_worst"] = float(np.max(np.abs(gE - oE) / (tau * (np.abs(oE) + bref)), initial=0.0))
    gG, oG = g["G"][gi][feas], o["G"][oi][feas]
    nG = np.linalg.norm(oG, axis=1)
    rep["G_pair_worst"] = float(np.max(np.linalg.norm(gG - oG, axis=1) / (tau * (nG + bref / w)), initial=0.0))
    ok = g["code"][gi][feas] == o["code"][oi][feas]  # where the sub-cases agree (else a boundary tie)
    gH, oH = g["Hpsd"][gi][feas][ok].reshape(-1, 144), o["Hpsd"][oi][feas][ok].reshape(-1, 144)
    nH = np.linalg.norm(oH, axis=1)
    rep["H_pair_worst"] = float(np.max(np.linalg.norm(gH - oH, axis=1) / (tau * (nH + bref[ok] / w[ok] ** 2)),
                                       initial=0.0))
    asm = oracle.assemble(o, nv)
    sig = float(np.sum(np.abs(oE) + bref))
    rep["E_total_worst"] = abs(g["E_total"] - asm["E"]) / (tau * sig) if np.isfinite(asm["E"]) else None
    verts = o["verts"][oi][feas]
    gb = np.zeros(nv)
    for q in range(4):
        np.add.at(gb, verts[:, q], tau * (nG + bref / w))
    dg = np.linalg.norm(g["g"] - asm["g"], axis=1)
    rep["g_worst"] = float(np.max(dg / np.maximum(gb, 1e-300), initial=0.0))
    rep["bsr_pattern_equal"] = bool(np.array_equal(g["row_ptr"], asm["row_ptr"]) and
                                    np.array_equal(g["col"], asm["col"]))
    if rep["bsr_pattern_equal"] and np.all(ok):
        nHall = np.linalg.norm(o["Hpsd"][oi][feas].reshape(-1, 144), axis=1)
        hb = np.zeros(nv)
        for q in range(4):
            np.add.at(hb, verts[:, q], tau * (nHall + bref / w ** 2))
        rows = np.repeat(np.arange(nv), np.diff(asm["row_ptr"]))
        dv = np.linalg.norm((g["val"] - asm["val"]).reshape(-1, 9), axis=1)
        rep["bsr_worst"] = float(np.max(dv / np.maximum(hb[rows], 1e-300), initial=0.0))
    return rep


# FP64 operations of additive CCD (model): per pair in the swept set (loads,
# mean displacement, motion bound, exact swept-box test, first distance,
# filter) and per step (position update, classification, gap)
ACCD_FLOPS_SETUP = 180.0
# per-kernel timing: launches captured back to back in one graph (replayed;
# a lone short kernel per replay would time the replay's launch instead)
KERNEL_LAUNCHES = 10
ACCD_FLOPS_PER_ITER = 110.0


def bench_linesearch(args):
    """One line-search pass of a Newton iteration (Sec. 3.3, last paragraph;
    App. A) per step: the broad phase over the boxes swept from x to x + p,
    additive CCD of every pair in the swept set with its filtered offset, and
    the energy alone at the step found (read on the device).  p is the seeded
    search direction of the workload (a squeeze toward the mid-plane plus
    noise, a few activation bands)."""
    import torch
    import synth
    import paper_2510_10256_amd as bfc

    sc = synth.workload(args.workload)
    p = synth.search_direction(sc)
    dev = torch.device("cuda:0")
    x = torch.tensor(sc.x, dtype=torch.float64, device=dev)
    pt = torch.tensor(p, dtype=torch.float64, device=dev)
    cs = bfc.ContactScene(sc, device=dev)
    cs.run(x)
    n_bp = cs.fit_swept(x, pt)
    tstep = torch.zeros(1, dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    def one_pass():
        cs.build_candidates_swept(x, pt)
        cs.max_step(x, pt, out=tstep)
        cs.eval_energy(x, pt, tstep, out=E)

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_start = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        one_pass()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = wall * 1e3 / args.steps
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    # the swept set and the step counts (one more max_step with per-pair output)
    t_dev, tp, it = cs.max_step(x, pt, per_pair=True)
    torch.cuda.synchronize()
    tp, it = tp[:n_bp].cpu().numpy(), it[:n_bp].cpu().numpy()
    n_ccd = int(np.sum(tp >= 0.0))
    iters = int(np.sum(it))
    # k_accd (with its final minimum) timed alone on the launching stream
    reps = max(20, args.steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cs.max_step(x, pt, out=tstep)
    e0.record(stream)
    for _ in range(reps):
        cs.max_step(x, pt, out=tstep)
    e1.record(stream)
    torch.cuda.synchronize()
    accd_ms = e0.elapsed_time(e1) / reps
    flops = n_ccd * ACCD_FLOPS_SETUP + iters * ACCD_FLOPS_PER_ITER
    roof = {"kernel": "k_accd (max_step_accd)", "bound": "alu", "achieved": flops / (accd_ms * 1e-3) / 1e12,
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": None, "kernel_ms": accd_ms,
            "units": {"ccd_pairs": n_ccd, "accd_steps": iters, "fp64_flops": flops}}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {
        "metric": "line search: CCD pairs/s (swept broad phase + additive CCD with filtered offsets + energy at the "
                  "step); p50/p99 latency",
        "value": n_ccd / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator and search direction)",
        "config": {"workload": f"{sc.name} line search", "n_verts": sc.n_verts, "N_bp_swept": n_bp,
                   "N_ccd": n_ccd, "accd_steps": iters, "step": float(t_dev.item()),
                   "energy_at_step": float(E.item())},
        "roofline": roof,
    }
    if args.cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        reps_c, t_total = 0, 0.0
        while t_total < 10.0 and reps_c < 20:
            t0 = time.perf_counter()
            r = oracle.max_step(sc, sc.x, p, nthreads=threads)
            oracle.energy(sc, sc.x + r["t"] * p, nthreads=threads)
            t_total += time.perf_counter() - t0
            reps_c += 1
        assert len(r["tpair"]) == n_ccd, (len(r["tpair"]), n_ccd)
        out["cpu_baseline"] = {"value": n_ccd * reps_c / t_total, "unit": "pairs/s", "cores": threads,
                               "kind": "oracle", "sample": f"whole workload, {reps_c} pass(es) of ACCD over the "
                                                           f"swept pair set and the energy at the step"}
    print(json.dumps(out))


def bench_locking(args):
    """Contact locking at rest (Fig. self_pushing_toy_example; App. A): a 5 cm
    straight rod (h = 300 um) and a 2 cm flat sheet (h = 1000 um) at rest, for
    several segment lengths, with the paper's filter, no filter and culling
    at 11 and 5 elements (rods).  Per case: pairs within h, active pairs,
    barrier energy and the largest vertex force at rest (all zero without
    locking), and the time of one step on the GPU."""
    import torch
    import synth
    import paper_2510_10256_amd as bfc

    dev = torch.device("cuda:0")
    modes = {"filter": (bfc.BF_FILTER_PAPER, 11), "none": (bfc.BF_FILTER_NONE, 11),
             "cull11": (bfc.BF_FILTER_CULL, 11), "cull5": (bfc.BF_FILTER_CULL, 5)}
    rows = []
    cases = [("rod", ell, synth.straight_rod(ell)) for ell in (1000.0, 600.0, 300.0, 200.0, 150.0, 100.0, 50.0, 25.0)]
    cases += [("sheet", ell, synth.flat_sheet(ell)) for ell in (2000.0, 1000.0, 700.0, 500.0, 350.0, 250.0)]
    for kind, ell, sc in cases:
        x = torch.tensor(sc.x, dtype=torch.float64, device=dev)
        for name, (mode, r) in modes.items():
            if kind == "sheet" and mode == bfc.BF_FILTER_CULL:
                continue
            cs = bfc.ContactScene(sc, filter_mode=mode, cull_radius=r, device=dev)
            cs.run(x)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                cs.step(x)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / 5
            c = cs.counts()
            gmax = float(cs.g.abs().max().item())
            rows.append({"kind": kind, "ell_um": ell, "h_um": sc.h, "eta_um": sc.eta, "mode": name,
                         "n_verts": sc.n_verts, "N_c": c["n_c"], "N_act": c["n_act"], "E_rest": float(cs.E.item()),
                         "max_vertex_force": gmax, "ms_per_step": ms})
            cs.close()
    locked = {m: [r["ell_um"] for r in rows if r["mode"] == m and r["N_act"] > 0] for m in modes}
    print(json.dumps({"metric": "contact locking at rest: active pairs, energy and largest vertex force per "
                                "resolution and mode (zero without locking)", "value": None, "unit": None,
                      "n_gpus": 1, "higher_is_better": None, "data": "synthetic (straight rod 5 cm, flat sheet 2 cm)",
                      "locked_resolutions_um": locked, "rows": rows}))


def bench_batch(args):
    """64 independent yarn / cloth patches (1k-64k primitives, log-uniform),
    stepped together by one graph launch."""
    import torch
    import synth
    import paper_2510_10256_amd as bfc

    prec_name = args.prec or "mixed"
    prec = bfc.BF_FP64 if prec_name == "fp64" else bfc.BF_MIXED
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    scenes = synth.batch_scenes()
    css, xs = [], []
    for sc in scenes:
        cs = bfc.ContactScene(sc, prec=prec, device=dev)
        x = torch.tensor(sc.x, dtype=torch.float64, device=dev)
        cs.run(x)
        if args.tune:
            cs.tune(x)
        css.append(cs)
        xs.append(x)
    counts = [cs.counts() for cs in css]
    n_c = sum(c["n_c"] for c in counts)
    n_act = sum(c["n_act"] for c in counts)
    stream = torch.cuda.current_stream(dev)
    # per-scene evaluation kernel times (eager, one scene at a time) for the roofline
    eval_ms, kinds = 0.0, []
    for cs, x, c in zip(css, xs, counts):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(5):
            e0.record(stream)
            cs.eval_barrier(x)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        eval_ms += float(np.median(ts))
        kinds.append(KIND_OF_CODE[cs.a_code[:c["n_act"]].cpu().numpy()])
    kinds = np.concatenate(kinds)

    def timed(batch, steps, warmup):
        for _ in range(warmup):
            batch.step()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t_start = time.perf_counter()
        ev[0].record(stream)
        for k in range(steps):
            batch.step()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return wall * 1e3 / steps, np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])

    seq = bfc.Batch(css, xs, lanes=1)
    seq_ms, _ = timed(seq, max(5, args.steps // 4), 2)
    seq.close()
    batch = bfc.Batch(css, xs, lanes=args.lanes)
    setup_s = time.perf_counter() - t0
    ms_per_step, step_ms = timed(batch, args.steps, args.warmup)
    for cs, c in zip(css, counts):
        st = cs.status(clear=True)
        assert not (st & (bfc.BF_S_CAND_OVERFLOW | bfc.BF_S_ACT_OVERFLOW | bfc.BF_S_BSR_OVERFLOW)), st
        assert cs.counts() == c
    out = {
        "metric": "filtered contact pairs evaluated/s (dist+filter+grad+Hessian); p50/p99 latency",
        "value": n_c / (ms_per_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "p50_ms": float(np.percentile(step_ms, 50)), "p99_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": "batch64: 64 yarn / cloth patches, 1k-64k primitives each (log-uniform), "
                               "one graph launch per step",
                   "scenes": len(css), "primitives": int(sum(sc.n_prims for sc in scenes)),
                   "N_c": n_c, "N_act": n_act, "lanes": batch.lanes,
                   "pq_choices": {str(q): int(sum(cs.pq == q for cs in css)) for q in (2, 4, 8, 16)},
                   "precision": prec_name},
        "active_pairs_per_s": n_act / (ms_per_step * 1e-3),
        "one_lane_ms_per_step": seq_ms,
        "setup_s": setup_s,
        "roofline": eval_roofline(eval_ms, n_act, kinds, "k_eval (eval_barrier), summed over the scenes", prec_name),
    }
    batch.close()
    if args.cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t_total, n_done, done = 0.0, 0, 0
        for sc, c in zip(scenes, counts):
            t1 = time.perf_counter()
            res = oracle.evaluate(sc, mode=1, derivs=True, nthreads=threads)
            t_total += time.perf_counter() - t1
            assert oracle.counts(res)["n_c"] == c["n_c"]
            n_done += c["n_c"]
            done += 1
            if t_total > 10.0:
                break
        out["cpu_baseline"] = {"value": n_done / t_total, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"the first {done} of the 64 scenes, one evaluation each"}
    print(json.dumps(out))


def _native_loop(sv, make, n, inflight, arrivals=None):
    """Requests through the library's serving loop: closed loop with `inflight`
    outstanding, or open loop at the given arrival times (s).  Returns the
    results (latency in ms, submit to completion) and the wall time."""
    pending, out = {}, []
    t0 = time.perf_counter()
    k = 0
    while k < n or pending:
        now = time.perf_counter() - t0
        while k < n and (len(pending) < inflight if arrivals is None else arrivals[k] <= now):
            r = make(k)
            pending[sv.submit(r.sid, r.x)] = r
            k += 1
        for t in list(pending):
            res = sv.poll(t, wait=False)
            if res is not None:
                pending.pop(t)
                out.append(res)
        if arrivals is not None and k < n and not pending:
            time.sleep(max(0.0, arrivals[k] - (time.perf_counter() - t0)))
        elif pending:
            time.sleep(20e-6)
    return out, time.perf_counter() - t0


def bench_serve_native(args):
    """The serving workload through the library's own loop (bf_serve_*):
    scenes created in device blocks of their own and evicted under the budget
    by the library; the same scenes, requests and load sweep as bench_serve."""
    import synth
    import paper_2510_10256_amd as bfc
    from paper_2510_10256_amd import serve
    from paper_2510_10256_amd.binding import NativeServer

    prec_name = args.prec or "mixed"
    prec = bfc.BF_FP64 if prec_name == "fp64" else bfc.BF_MIXED
    scenes = synth.serving_scenes()
    budget_gib = 4.0 if args.budget_gib is None else args.budget_gib
    budget = int(budget_gib * (1 << 30))
    caps = [serve.scene_caps(sc) for sc in scenes]
    sv = NativeServer(scenes, caps, budget_bytes=budget, slots=args.slots, prec=prec)
    make = serve.request_maker(scenes, seed=4242)
    lbar = [serve.mean_edge_length(sc) for sc in scenes]

    def first_touch(k):  # one request per scene: every scene made resident (as far as the budget allows)
        rng = np.random.default_rng(77 + k)
        return serve.Request(rid=-1 - k, sid=k, x=scenes[k].x + rng.normal(0.0, 0.01 * lbar[k], scenes[k].x.shape))

    t0 = time.perf_counter()
    _native_loop(sv, first_touch, len(scenes), 2 * args.slots)  # warm-up: scene creation
    setup_s = time.perf_counter() - t0
    ev0 = sv.info()
    done, wall = _native_loop(sv, lambda k: make(1000 + k), args.requests, 2 * args.slots)
    sat_rate = len(done) / wall
    sat_pairs = sum(r["counts"]["n_c"] for r in done) / wall
    ev1 = sv.info()
    runs = {}
    for frac in (0.25, 0.5, 0.75, 0.9):
        n = args.requests if frac == 0.75 else max(60, args.requests // 3)
        arr = serve.poisson_arrivals(frac * sat_rate, n, seed=int(frac * 100))
        e0 = sv.info()
        d, w = _native_loop(sv, lambda k, f=frac: make(int(f * 1e6) + k), n, 0, arrivals=arr)
        e1 = sv.info()
        lat = np.array([r["ms"] for r in d])
        runs[str(frac)] = {"rate_req_s": frac * sat_rate, "requests": n,
                           "pairs_per_s": sum(r["counts"]["n_c"] for r in d) / w,
                           "mean_ms": float(lat.mean()), "p50_ms": float(np.percentile(lat, 50)),
                           "p99_ms": float(np.percentile(lat, 99)),
                           "errors": int(sum(r["error"] != 0 for r in d)),
                           "overflow": int(sum((r["status"] & 0x1b) != 0 for r in d)),
                           "scenes_created": e1["created"] - e0["created"],
                           "scenes_evicted": e1["evicted"] - e0["evicted"],
                           "retries": int(sum(r["retries"] for r in d))}
    info = sv.info()
    sv.close()
    head = runs["0.75"]
    out = {
        "metric": "filtered contact pairs evaluated/s (dist+filter+grad+Hessian); p50/p99 latency",
        "value": head["pairs_per_s"], "unit": "pairs/s",
        "n_gpus": 1, "steps": head["requests"], "warmup": 32, "ms_per_step": head["mean_ms"],
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": "serve256 through the library's serving loop (bf_serve_*): 256 rod / shell scenes "
                               "(1:1, lognormal sizes, median 16k primitives), Poisson arrivals at 0.75 of "
                               f"saturation, HBM budget {budget_gib:g} GiB (resident scenes and running steps), "
                               f"{args.slots} slots",
                   "scenes": len(scenes), "primitives": int(sum(sc.n_prims for sc in scenes)),
                   "budget_bytes": budget, "slots": args.slots, "precision": prec_name,
                   "resident_at_end": info["resident"], "footprint_median_bytes": int(np.median(info["footprint"]))},
        "saturation": {"req_per_s": sat_rate, "pairs_per_s": sat_pairs, "requests": len(done),
                       "scenes_created": ev1["created"] - ev0["created"]},
        "sweep": runs,
        "setup_s": setup_s,
        "scenes_created": info["created"], "scenes_evicted": info["evicted"], "overflow_reruns": info["retried"],
        "peak_bytes_in_use": info["peak_bytes"], "largest_step_bytes": int(info["step"].max()),
        "resident_bytes_all_scenes": int(info["footprint"].sum()),
        "roofline": None,
    }
    print(json.dumps(out))


def bench_serve(args):
    """Serving loop: 256 resident rod / shell scenes (lognormal sizes), Poisson
    arrivals, admission by HBM budget; p50/p99 latency and pairs/s at 0.75 of
    the measured saturation rate, plus a sweep of the load."""
    import torch
    import synth
    import paper_2510_10256_amd as bfc
    from paper_2510_10256_amd import serve

    prec_name = args.prec or "mixed"
    prec = bfc.BF_FP64 if prec_name == "fp64" else bfc.BF_MIXED
    scenes = synth.serving_scenes()
    budget_gib = 2.0 if args.budget_gib is None else args.budget_gib
    budget = int(budget_gib * (1 << 30))
    server = serve.Server(scenes, budget_bytes=budget, slots=args.slots, prec=prec)
    make = serve.request_maker(scenes, seed=4242)
    t0 = time.perf_counter()
    serve.run_closed_loop(server, make, n_requests=32, inflight=2 * args.slots)  # warm-up
    done, wall = serve.run_closed_loop(server, lambda k: make(1000 + k), n_requests=args.requests,
                                       inflight=2 * args.slots)
    sat_rate = len(done) / wall
    sat_pairs = sum(r.counts["n_c"] for r in done) / wall
    runs = {}
    for frac in (0.25, 0.5, 0.75, 0.9):
        n = args.requests if frac == 0.75 else max(60, args.requests // 3)
        arr = serve.poisson_arrivals(frac * sat_rate, n, seed=int(frac * 100))
        c0, e0 = server.created, server.evicted
        d, w = serve.run_open_loop(server, lambda k, f=frac: make(int(f * 1e6) + k), arr)
        st = serve.latency_stats(d)
        runs[str(frac)] = {"rate_req_s": frac * sat_rate, "requests": n, "pairs_per_s":
                           sum(r.counts["n_c"] for r in d) / w, **st, "scenes_created": server.created - c0,
                           "scenes_evicted": server.evicted - e0, "retries": int(sum(r.retries for r in d))}
    head = runs["0.75"]
    out = {
        "metric": "filtered contact pairs evaluated/s (dist+filter+grad+Hessian); p50/p99 latency",
        "value": head["pairs_per_s"], "unit": "pairs/s",
        "n_gpus": 1, "steps": head["requests"], "warmup": 32, "ms_per_step": head["mean_ms"],
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": "serve256: 256 resident rod / shell scenes (1:1, lognormal sizes, median 16k "
                               "primitives), Poisson arrivals at 0.75 of saturation, HBM budget "
                               f"{budget_gib:g} GiB, {args.slots} slots",
                   "scenes": len(scenes), "primitives": int(sum(sc.n_prims for sc in scenes)),
                   "budget_bytes": budget, "slots": args.slots, "precision": prec_name},
        "saturation": {"req_per_s": sat_rate, "pairs_per_s": sat_pairs, "requests": len(done)},
        "sweep": runs,
        "setup_s": time.perf_counter() - t0,
        "roofline": None,
    }
    server.close()
    if args.cpu_baseline:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t_total, n_done, k = 0.0, 0, 0
        while t_total < 10.0 and k < 64:
            req = make(5000 + k)
            sc = scenes[req.sid].with_positions(req.x)
            t1 = time.perf_counter()
            res = oracle.evaluate(sc, mode=1, derivs=True, nthreads=threads)
            t_total += time.perf_counter() - t1
            n_done += oracle.counts(res)["n_c"]
            k += 1
        out["cpu_baseline"] = {"value": n_done / t_total, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"{k} requests of the same stream, one evaluation each"}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this path runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.path == "locking":
        return bench_locking(args)
    if args.path == "linesearch":
        if args.workload in ("batch64", "serve256"):
            print("bench.py: the line-search pass runs on one scene (woven_patch, folded_cloth, helix_loop_rod)",
                  file=sys.stderr)
            sys.exit(2)
        return bench_linesearch(args)
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "serve256":
        return bench_serve_native(args) if args.native_serve else bench_serve(args)
    import torch
    import synth
    import paper_2510_10256_amd as bfc

    args.prec = args.prec or "fp64"
    sc = synth.workload(args.workload)
    prec = bfc.BF_FP64 if args.prec == "fp64" else bfc.BF_MIXED
    dev = torch.device("cuda:0")
    x_np = sc.x * np.array([1.0, 1.0, args.core_squeeze]) if args.core_squeeze > 0 else sc.x
    x = torch.tensor(x_np, dtype=torch.float64, device=dev)
    cs = bfc.ContactScene(sc, prec=prec, device=dev)
    t0 = time.perf_counter()
    cs.run(x)  # sizes the buffers (grows them on overflow, then steps again)
    n_core = 0
    if args.core_squeeze > 0:  # the temporary zero offset of the pairs inside the core (Sec. 3.4)
        cs.build_candidates(x)
        n_core = int(cs.core_mark(x).item())
        cs.run(x)
    if args.tune:
        cs.tune(x)  # threads per broad-phase query
        cs.run(x)
    fric = args.friction_mu > 0
    if fric:  # lagged friction (App. A): the active list and its data at the previous positions
        xlag_np = x_np - 0.02 * synth.search_direction(sc)
        xlag = torch.tensor(xlag_np, dtype=torch.float64, device=dev)
        cs.run(xlag)
        cs.friction_lag(xlag)
        cs.run(x)
        n_fric = int(cs.f_cnt.item())
    counts = cs.counts()
    n_c, n_act = counts["n_c"], counts["n_act"]
    codes = cs.a_code[:n_act].cpu().numpy()
    kinds = KIND_OF_CODE[codes]

    stream = torch.cuda.current_stream(dev)

    def step():
        cs.step(x)
        if fric:
            cs.friction_eval(x, args.friction_mu, args.eps_vh)
            cs.friction_assemble()

    graph = None
    if args.graph != 0:
        # one step captured as a graph (every launch is on the current stream,
        # no host synchronisation and no allocation inside the step)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            step()
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()

    if args.copy_mib > 0:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE counters convert
        # the counters of the path's kernels to bytes
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed(use_graph):
        """W warm-up steps, then K timed steps (wall clock and per-step events)."""
        def one_step():
            if use_graph:
                graph.replay()
            else:
                step()
        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        ev[0].record(stream)
        for k in range(args.steps):
            one_step()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return wall * 1e3 / args.steps, np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]), wall

    # graph replay, and eager launches (where the assembly's structure runs
    # on the scene's second stream beside the evaluation kernel)
    modes = {}
    if args.graph != 0:
        modes["graph"] = timed(True)
    if args.graph != 1:
        modes["eager"] = timed(False)
    launch = min(modes, key=lambda m: modes[m][0])
    ms_per_step, step_ms, wall = modes[launch]
    st = cs.status(clear=True)
    assert not (st & (bfc.BF_S_CAND_OVERFLOW | bfc.BF_S_ACT_OVERFLOW | bfc.BF_S_BSR_OVERFLOW)), st
    assert cs.counts() == counts, (cs.counts(), counts)

    # per-call durations on the launching stream (eager, after the timed region)
    calls = ["build_candidates", "filter_pairs", "eval_barrier", "assemble_grad_hess"]
    fns = [lambda: cs.build_candidates(x), lambda: cs.filter_pairs(x), lambda: cs.eval_barrier(x),
           lambda: cs.assemble_grad_hess()]
    if fric:
        calls += ["friction_eval", "assemble_grad_hess (friction)"]
        fns += [lambda: cs.friction_eval(x, args.friction_mu, args.eps_vh), lambda: cs.friction_assemble()]
    per = {c: [] for c in calls}
    for _ in range(max(10, args.steps // 5)):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
        e[0].record(stream)
        for q, f in enumerate(fns):
            f()
            e[q + 1].record(stream)
        torch.cuda.synchronize()
        for q, c in enumerate(calls):
            per[c].append(e[q].elapsed_time(e[q + 1]))
    call_ms = {c: float(np.mean(v)) for c, v in per.items()}

    # per-stage kernel durations: HIP events around each stage's kernels on
    # the stream they run on (the library's stage timers), eager steps after
    # the timed region; medians over the steps
    cs.set_timing(True)
    stage_runs = []
    for _ in range(max(10, args.steps // 5)):
        cs.step(x)
        stage_runs.append(cs.stage_ms())
    cs.set_timing(False)
    stage_ms = {k: float(np.median([r[k] for r in stage_runs])) for k in stage_runs[0]}
    step_roof = step_roofline(sc, counts, kinds, stage_ms, ms_per_step, args.prec)
    roof = dict(step_roof["dominant"])
    roof["step"] = {k: v for k, v in step_roof.items() if k != "dominant"}
    fric_roof = None
    if fric:
        # friction_eval alone (one kernel): ten launches captured back to back in
        # one graph, replays timed with events on the launching stream
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            cs.friction_eval(x, args.friction_mu, args.eps_vh)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            for _ in range(10):
                cs.friction_eval(x, args.friction_mu, args.eps_vh)
        torch.cuda.synchronize()
        reps = max(4, args.steps // 10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g.replay()
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        f_ms = e0.elapsed_time(e1) / (reps * 10)
        fb = float(friction_bytes_per_pair(args.prec) * n_fric)
        fric_roof = {"kernel": "k_friction_eval (friction_eval)", "bound": "hbm",
                     "achieved": fb / (f_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None,
                     "kernel_ms": f_ms, "units": {"lagged_pairs": n_fric, "bytes": fb}}
        fric_roof["frac"] = fric_roof["achieved"] / HBM_PEAK_GBS
        if (args.core_squeeze == 0 and args.prec != "mixed" and sc.name in FRICTION_TRAFFIC_BYTES
                and friction_source_fingerprint() == FRICTION_TRAFFIC_SOURCE):
            fric_roof["traffic"] = FRICTION_TRAFFIC_BYTES[sc.name]
    key = (roof["stage"], sc.name, args.prec)
    if args.core_squeeze == 0 and not fric and key in TRAFFIC:
        src, per_launch = TRAFFIC[key]
        if stage_source_fingerprint(roof["stage"]) == src:
            roof["traffic"] = per_launch

    out = {
        "metric": "filtered contact pairs evaluated/s (dist+filter+grad+Hessian"
                  + (" + lagged friction" if fric else "") + "); p50/p99 latency",
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
        "dtype": "f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": f"{sc.name}: " + ("32 warp x 32 weft rods, 512 vertices per rod, segments "
                                                 "20-300 um, h = 300 um, dhat = 30 um"
                                                 if sc.name == "woven_patch" else sc.name)
                               + (f"; z scaled by {args.core_squeeze}, pairs inside the core under the temporary "
                                  f"zero offset" if args.core_squeeze > 0 else "")
                               + (f"; lagged friction mu = {args.friction_mu}, eps_vh = {args.eps_vh} um"
                                  if fric else ""),
                   "n_verts": sc.n_verts, "n_edges": sc.n_edges, "n_tris": sc.n_tris,
                   "N_bp": counts["n_bp"], "N_c": n_c, "N_filt": counts["n_filt"], "N_act": n_act,
                   "nnzb": counts["nnzb"], "launch": launch, "pq": cs.pq, "precision": args.prec,
                   "N_band": cs.deferred()[0], "N_exact": cs.deferred()[1],
                   **({"N_friction": n_fric} if fric else {}),
                   **({"core_squeeze_z": args.core_squeeze, "core_pairs_marked": n_core,
                       "core_pairs_live": int(cs.core_live().item())} if args.core_squeeze > 0 else {})},
        "active_pairs_per_s": n_act / (ms_per_step * 1e-3),
        "call_ms": call_ms,
        "launch": launch,
        "ms_per_step_by_launch": {m: v[0] for m, v in modes.items()},
        "setup_s": time.perf_counter() - t0 - sum(v[2] for v in modes.values()),
        "roofline": roof,
        **({"friction_roofline": fric_roof} if fric else {}),
    }
    if args.cpu_baseline:
        core = None
        if args.core_squeeze > 0:
            import oracle
            core = oracle.core_mark(sc, x_np)
        fr = None
        if fric:
            import oracle
            fr = (oracle.friction_lag(sc, xlag_np), xlag_np, args.friction_mu, args.eps_vh)
        out["cpu_baseline"], res = cpu_baseline(sc, n_c, x_np if (args.core_squeeze > 0 or fric) else None, core, fr)
        # the error of every result of the step against the oracle's, on the whole workload
        g = cs.results()
        del g["cand"]
        out["oracle_errors"] = oracle_errors(g, res, sc.n_verts, sc.kappa, 1e-10 if args.prec == "fp64" else 1e-5)
        del g, res
    print(json.dumps(out))


if __name__ == "__main__":
    main()
