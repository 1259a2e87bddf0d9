#!/usr/bin/env python3
"""Throughput of the colour-coding hot path on one MI355X, in colour-set-edge updates per second.

One step = one pass of the whole hot path over one batch of synthetic input: colour the graph
B times (B = the workload's colourings per batch), then run the full dynamic program for every
colouring (all template splits: neighbour gather + combine, cut-row finish, root sum).

Units (CSEU): for a split whose passive sub-template has p vertices, every directed CSR entry
accounts for C(k, p) colour-set updates (1 when p = 1), summed over the splits of the template's
reference partition (root at the centre). units per step = nnz * units_per_edge * B.

Usage:
  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
  python bench.py --summarize-pmc DIR ...   (turn rocprofv3 --pmc output into profiles/*.json)

Prints one JSON line (rank 0). Only one GPU is used: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "colour-set·edge updates/s (u12, RMAT-23) plain vs batched; p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1804_09764_amd", "csrc", "cc_kernels.hip")

WORKLOADS = {
    # R-MAT (a, b, c) = (0.57, 0.19, 0.19), symmetrised, de-duplicated; 12-vertex Pruefer tree
    "rmat20-ef16-u12": dict(scale=20, ef=16, gseed=1, k=12, tseed=12, B=1, trust=False),
    "rmat23-ef256-u12": dict(scale=23, ef=256, gseed=3, k=12, tseed=12, B=4, trust=True),
    "rmat20-ef16-u15": dict(scale=20, ef=16, gseed=1, k=15, tseed=15, B=1, trust=False),
    # a 15-vertex tree whose live tables exceed HBM (counted with --only-budget)
    "rmat22-ef16-u15": dict(scale=22, ef=16, gseed=1, k=15, tseed=2, B=1, trust=True),
}
DEFAULT_WORKLOAD = "rmat23-ef256-u12"


def _code_only(text: str) -> str:
    """C/C++ source without comments and blank lines (the sources hold no string literal with a
    comment marker), so that edits to comments keep the hash."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_hash(workload: str = DEFAULT_WORKLOAD) -> str:
    """Hash of what fixes the split kernel's memory accesses on a workload: the kernel's code
    (comments excluded) and the device constants the planner writes for the workload's template
    (row storage order, split lists, fold maps, masks), read back through cc_plan_constants_get."""
    import inputs
    import paper_1804_09764_amd as cc
    W = WORKLOADS[workload]
    h = hashlib.sha256(_code_only(open(KERNEL_SRC).read()).encode())
    h.update(cc.Plan(inputs.pruefer_tree(W["k"], W["tseed"]), bind=False).constants().tobytes())
    return h.hexdigest()[:16]


def reference_plan_model(T, nnz, colourings, seconds):
    """The reference partition (centre root, cut smallest child) behind the CSEU units, and two
    figures reported beside them, never mixed with them: the combine's multiply-adds per vertex,
    sum over splits of C(k, s) C(s, a), and the paper's per-neighbour cost model, the same sum per
    CSR entry (C(k, |T_i|) C(|T_i|, |T_i'|) per split, Section 3.2), as operations per second."""
    import paper_1804_09764_amd as cc
    ref = cc.Plan(T, flags=cc.CC_PLAN_CENTRE_SMALLEST, bind=False)
    k = ref.k
    fma = sum(math.comb(k, s) * math.comb(s, a) for (s, a, _) in ref.splits)
    return {"splits": [list(x) for x in ref.splits], "units_per_edge": ref.info.units_per_edge,
            "combine_fma_per_vertex": fma, "paper_model_ops_per_edge": fma,
            "paper_model_ops_per_s": float(nnz) * fma * colourings / seconds}


def widths(k, s, a, p):
    W = lambda t: math.comb(k - 1, t - 1)  # noqa: E731  colour-anchored row width
    return W(p), W(a), W(s)


def split_bytes(k, s, a, p, n, nnz):
    """Compulsory HBM bytes of one split's gather+combine launch: every array crosses HBM once.

    CSR columns (4 B per entry) and row offsets (8 B per vertex), colours (1 B per vertex), the
    passive table when p >= 2 (8 B per vertex per column), the active table when a >= 2, and the
    output table, all in the colour-anchored widths.
    """
    Wp, Wa, Ws = widths(k, s, a, p)
    b = 4 * nnz + 8 * (n + 1) + n
    if p >= 2:
        b += 8 * n * Wp
    if a >= 2:
        b += 8 * n * Wa
    b += 8 * n * Ws
    return b


def needed_lines(k, p):
    """Expected number of 128-byte lines of a neighbour's colour-anchored passive row that hold at
    least one entry the row needs. The row lists the (p-1)-sets over the neighbour's k-1 other
    colours in the library's storage order (cc_entry_order), 16 entries per line; an entry is
    needed unless its set holds the row's colour, whose position among those k-1 colours is
    uniform."""
    K = k - 1
    colex = [m for m in range(1 << K) if bin(m).count("1") == p - 1]  # colex = increasing order
    W = len(colex)
    if W <= 16:
        return 1.0
    import paper_1804_09764_amd as cc
    masks = [colex[r] for r in cc.entry_order(k, p - 1)]
    total = 0
    for x in range(K):
        total += sum(1 for l in range(0, W, 16) if any(not (masks[j] >> x) & 1 for j in range(l, min(l + 16, W))))
    return total / K


def method_bytes(k, s, a, p, n, nnz):
    """Bytes the method must move for one split launch, counting only the values the arithmetic
    uses. Per CSR entry: the neighbour's colour (1 B, from the per-entry colour array the count
    gathers once per colouring), the column (4 B, when p >= 2) and, for the expected fraction
    (k-1)/k of neighbours whose colour differs from the row's, the C(k-2, p-1) entries of the
    neighbour's colour-anchored passive row whose set avoids the row's colour (8 B each; the
    other entries of that row add to sets no term of the combine reads). Per vertex: its row
    offsets, colour, active row (a >= 2) and output row."""
    Wp, Wa, Ws = widths(k, s, a, p)
    b = (5 if p >= 2 else 1) * nnz + 8 * (n + 1) + n + 8 * n * Ws + (8 * n * Wa if a >= 2 else 0)
    if p >= 2:
        b += 8 * math.comb(k - 2, p - 1) * nnz * (k - 1) / k
    return b


def method_bytes_packed(k, s, a, p, n, nnz, B):
    """method_bytes for a packed launch of B colourings: per CSR entry the column, the neighbour's
    B colours and the needed passive entries of each colouring; per vertex B colours, B active rows
    (a >= 2) and B output rows."""
    Wp, Wa, Ws = widths(k, s, a, p)
    b = (4 + B) * nnz + 8 * (n + 1) + B * n + 8 * B * n * Ws + (8 * B * n * Wa if a >= 2 else 0)
    if p >= 2:
        b += 8 * B * math.comb(k - 2, p - 1) * nnz * (k - 1) / k
    return b


def loaded_bytes_projected(k, s, a, p, n, nnz, classes):
    """loaded_bytes for a split on projected passive rows (classes colour classes per pass): per CSR
    entry the neighbour's colour and column and, for the fraction (k-1)/k of neighbours whose colour
    differs from the row's, its projected row (C(k-2, p-1) entries padded to whole 128-byte
    lines); per vertex the same as loaded_bytes; plus the copies: every pass reads the table once
    and every vertex writes one projected row per colour other than its own."""
    Wp, Wa, Ws = widths(k, s, a, p)
    wn_pad = (math.comb(k - 2, p - 1) + 15) // 16 * 16
    wp_pad = (Wp + 15) // 16 * 16
    passes = -(-k // classes)
    b = 5 * nnz + 8 * (n + 1) + n + 8 * n * Ws + (8 * n * Wa if a >= 2 else 0)
    b += 8 * wn_pad * nnz * (k - 1) / k
    b += passes * 8 * n * wp_pad + (k - 1) * 8 * n * wn_pad
    return b


def loaded_bytes(k, s, a, p, n, nnz):
    """Algorithmic bytes of one split launch: what its loads and stores must move from HBM at the
    128-byte line granularity of the layout. Per CSR entry: the neighbour's colour (1 B, from the
    per-entry colour array the count gathers once per colouring), the column (4 B, when p >= 2) and,
    for the expected fraction (k-1)/k of neighbours whose colour differs from the row's, the lines
    of the neighbour's colour-anchored passive row that hold an entry the row needs (entries whose
    set holds the row's colour are skipped); per vertex: its row offsets, colour, active row
    (a >= 2) and output row."""
    Wp, Wa, Ws = widths(k, s, a, p)
    b = (5 if p >= 2 else 1) * nnz + 8 * (n + 1) + n + 8 * n * Ws + (8 * n * Wa if a >= 2 else 0)
    if p >= 2:
        b += 128 * needed_lines(k, p) * nnz * (k - 1) / k
    return b


def loaded_bytes_packed(k, s, a, p, n, nnz, B):
    """Algorithmic bytes of one packed launch (all B colourings of a split at once): per CSR entry
    the column (4 B), the neighbour's B colours (B bytes) and, when p >= 2, the neighbour's tile
    rows of 8 B C(k-1, p-1) per colouring, read for the fraction (k-1)/k of colourings in which
    the neighbour's colour differs from the row's; per vertex its row offsets, B colours, B active
    rows (a >= 2) and B output rows."""
    Wp, Wa, Ws = widths(k, s, a, p)
    b = (4 + B) * nnz + 8 * (n + 1) + B * n + 8 * B * n * Ws + (8 * B * n * Wa if a >= 2 else 0)
    if p >= 2:
        b += 8 * B * Wp * nnz * (k - 1) / k
    return b


def packed_kernel_split(k, s, a, p):
    """Whether a packed count runs this split on packed rows (every per-colouring width <= 64) or
    colouring by colouring with the one-colouring kernels."""
    Wp, Wa, Ws = widths(k, s, a, p)
    return (p < 2 or Wp <= 64) and Wa <= 64 and Ws <= 64


def load_traffic(workload: str, split_index: int):
    """HBM traffic per launch (GB) of the dominant kernel from committed rocprofv3 counters, or None
    if they were taken on another kernel source."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash(workload) or d.get("split_index") != split_index:
        return None
    return d["traffic_bytes_per_launch"] / 1e9


def cpu_baseline(row_ptr, col, T, target_s=15.0):
    """The oracle, timed on a bounded sample of the same workload.

    For every split of the reference partition, oracle.step (Eq. 1 as written: per vertex, per
    colour set, neighbours then splits) runs over a uniform random sample of centre vertices of the
    benchmark graph, with their true neighbour lists; the neighbours' passive rows come from a
    bounded table of random integers (row = neighbour id mod 65536) and the active rows are random
    integers. CSEU are counted exactly as on the GPU (deg(v) * w(p) per sampled vertex). The sample
    is doubled until it takes about `target_s` seconds.
    """
    import numpy as np

    import oracle
    import paper_1804_09764_amd as cc

    ref = cc.Plan(T, flags=cc.CC_PLAN_CENTRE_SMALLEST, bind=False)
    k = ref.k
    n = len(row_ptr) - 1
    rng = np.random.default_rng(2024)
    deg = np.diff(row_ptr)
    rows = 65536
    tables = {p: rng.integers(0, 4, size=(rows, math.comb(k, p))).astype(np.float64)
              for p in sorted({p for _, _, p in ref.splits})}

    def run(m):
        vs = np.sort(rng.choice(n, size=m, replace=False))
        lens = deg[vs]
        nbr_ptr = np.zeros(m + 1, dtype=np.int64)
        nbr_ptr[1:] = np.cumsum(lens)
        idx = (np.concatenate([col[row_ptr[v]:row_ptr[v + 1]] for v in vs]) if m else np.zeros(0, np.int32))
        idx = (idx % rows).astype(np.int32)
        units = 0
        secs = 0.0
        for (s, a, p) in ref.splits:
            act = rng.integers(0, 4, size=(m, math.comb(k, a))).astype(np.float64)
            t0 = time.perf_counter()
            oracle.step(k, s, a, nbr_ptr, idx, act, tables[p])
            secs += time.perf_counter() - t0
            units += int(lens.sum()) * (math.comb(k, p) if p >= 2 else 1)
        return units, secs, m

    m = 16
    units, secs, m = run(m)
    while secs < target_s / 2 and m < n:
        m = min(n, int(m * max(2.0, min(8.0, target_s / max(secs, 1e-3)))))
        units, secs, m = run(m)
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": units / secs, "unit": "CSEU/s", "cores": oracle.threads(), "kind": "oracle",
            "cpu_model": cpu_model, "host_cpus_visible": os.cpu_count(),
            "sample": f"{m} uniformly sampled centre vertices with their neighbour lists, every split of the "
                      f"reference partition, random integer tables (passive rows: 65536, indexed by neighbour id "
                      f"mod 65536); {units:.3e} CSEU in {secs:.1f} s"}


def bench(args):
    import numpy as np
    import torch

    import inputs
    import paper_1804_09764_amd as cc

    W = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    t0 = time.time()
    rp_d, col_d = inputs.rmat_graph_gpu(W["scale"], W["ef"], W["gseed"], device=dev)
    n, nnz = rp_d.numel() - 1, col_d.numel()
    print(f"[bench] graph scale={W['scale']} ef={W['ef']} n={n} nnz={nnz} built on the GPU in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    T = inputs.pruefer_tree(W["k"], W["tseed"])
    k, B = W["k"], W["B"]
    P = cc.Plan(T)
    tuned = None
    if args.autotune:
        # degree-split parameters by measurement (one colouring per candidate), before timing
        from paper_1804_09764_amd import autotune
        rec = autotune.tune(P, rp_d, col_d, seed=args.seed, cache_path=args.autotune, trust=W["trust"])
        args.hub_threshold, args.chunk = rec.hub_threshold, rec.chunk
        tuned = {"hub_threshold": rec.hub_threshold, "chunk": rec.chunk, "ms": rec.ms, "default_ms": rec.default_ms}
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
    G = cc.Graph(rp_d, col_d, hub_threshold=args.hub_threshold, chunk=args.chunk, trust=W["trust"])
    units_per_edge = P.info.units_per_edge
    ws = cc.Workspace()
    colours = torch.empty((B, n), dtype=torch.uint8, device=dev)
    X = torch.empty(B, dtype=torch.float64, device=dev)
    ws_bytes = cc.count_workspace_bytes(P, G)
    proj = cc.count_projection(P, G)
    print(f"[bench] plan root={P.info.root} splits={P.splits} workspace={ws_bytes / 1e9:.2f} GB "
          f"graph={G.info} projected classes per pass={proj}", file=sys.stderr, flush=True)
    if args.dispatch_map:
        # the dominant split: the one whose passive rows are the widest (ties: the later split)
        widths_p = [math.comb(k - 1, p - 1) if p >= 2 else 0 for (_, _, p) in P.splits]
        dom_split = max(range(len(widths_p)), key=lambda i: (widths_p[i], i))
        json.dump({"sequence": dispatch_sequence(P, G, proj), "dominant_split": dom_split},
                  open(args.dispatch_map, "w"))

    packed = args.path in ("packed", "auto")
    pack = B
    if packed:
        # colourings per packed count: all of the step's if their tables fit in HBM next to the
        # graph, else the largest power-of-two share that does (the counts run one after another
        # and reuse the workspace)
        free = torch.cuda.mem_get_info(dev)[0]
        while pack > 1 and cc.count_packed_workspace_bytes(P, G, pack) > 0.85 * free:
            pack //= 2
        if args.path == "auto" and (pack < B or B < 8):
            # packed rows pay off from about 8 colourings per count; below that, and when the
            # step's colourings do not fit in one packed count, the one-colouring path is faster
            packed = False
            ws_bytes = cc.count_workspace_bytes(P, G)
        else:
            ws_bytes = cc.count_packed_workspace_bytes(P, G, pack)
            print(f"[bench] packed counts of {pack} colourings, workspace {ws_bytes / 1e9:.2f} GB",
                  file=sys.stderr, flush=True)

    def step(i):
        cc.colour(G, k, seed=args.seed, first_iter=i * B, B=B, out=colours)
        if packed:
            for c0 in range(0, B, pack):
                cc.count_packed(P, G, colours[c0:c0 + pack], workspace=ws, out=X[c0:c0 + pack])
        else:
            cc.count(P, G, colours, workspace=ws, out=X)

    X0 = None  # the counts of the first warm-up step's colourings (the packed leg's reference)
    for i in range(args.warmup):
        step(i)
        if i == 0:
            X0 = X.clone()
    torch.cuda.synchronize()
    P.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
        if args.progress:
            torch.cuda.synchronize()
            print(f"[bench] step {i + 1}/{args.steps} done at {time.perf_counter() - t_start:.1f}s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    gather_ms, finish_ms, launches = P.profile_read()
    P.profile(False)
    Xh = X.cpu().numpy()

    units = float(nnz) * units_per_edge * B * args.steps
    value = units / elapsed
    dom = int(np.argmax(gather_ms))
    s, a, p = P.splits[dom]
    avg_ms = gather_ms[dom] / max(1, launches[dom])
    dom_packed = packed and packed_kernel_split(k, s, a, p)
    alg = method_bytes_packed(k, s, a, p, n, nnz, pack) if dom_packed else method_bytes(k, s, a, p, n, nnz)
    if dom_packed:
        lines = loaded_bytes_packed(k, s, a, p, n, nnz, pack)
    elif proj[dom] > 0:
        lines = loaded_bytes_projected(k, s, a, p, n, nnz, proj[dom])
    else:
        lines = loaded_bytes(k, s, a, p, n, nnz)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = None if dom_packed else load_traffic(args.workload, dom)
    per_split = [{"s": S, "a": A, "p": Pp, "gather_ms": round(float(g) / max(1, c), 4),
                  "finish_ms": round(float(f) / max(1, c), 4)}
                 for (S, A, Pp), g, f, c in zip(P.splits, gather_ms, finish_ms, launches)]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "CSEU/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": f"R-MAT scale {W['scale']} edge factor {W['ef']} "
                   f"(a,b,c)=(0.57,0.19,0.19) seed {W['gseed']}", "n": n, "nnz": nnz,
                   "template": f"Pruefer tree k={k} seed {W['tseed']}", "colourings_per_step": B,
                   "units_per_edge": units_per_edge, "path": "packed" if packed else "plain",
                   "colourings_per_packed_count": pack if packed else None,
                   "workspace_GB": ws_bytes / 1e9,
                   "degree_split": {"hub_threshold": G.info["hub_threshold"], "chunk": G.info["chunk"],
                                    "autotuned": tuned}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "traffic_unit": "GB per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by what they "
                                     "read for a 1 GiB device copy. These count L2-to-fabric requests, "
                                     "Infinity Cache hits included: an upper bound of the DRAM bytes, not "
                                     "a DRAM measurement",
                     "kernel": (f"k_psplit split {dom} (s={s}, a={a}, p={p})" if dom_packed else
                                f"k_project + k_split split {dom} (s={s}, a={a}, p={p}), projected rows, "
                                f"{proj[dom]} colour classes per pass" if proj[dom] > 0 else
                                f"k_split split {dom} (s={s}, a={a}, p={p})"),
                     "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": alg,
                     "algorithmic_bytes": "method bytes: only the passive entries the combine uses "
                                          "(bench.py method_bytes)",
                     "line_bytes_per_launch": lines,
                     "line_GBps": lines / (avg_ms * 1e-3) / 1e9,
                     "line_bytes": "the 128-byte lines holding a needed entry, plus the row copies of a "
                                   "projected split (bench.py loaded_bytes, loaded_bytes_projected)",
                     "compulsory_bytes_per_launch": split_bytes(k, s, a, p, n, nnz),
                     "traffic_GBps": (traffic / (avg_ms * 1e-3)) if traffic else None,
                     "traffic_over_method": (traffic * 1e9 / alg) if traffic else None},
        "splits": per_split,
        "reference_plan": reference_plan_model(T, nnz, B * args.steps, elapsed),
        "X_last": [float(x) for x in Xh],
    }
    if args.budget_frac > 0:
        out["budget"] = budget_leg(P, G, k, args, cc.count_workspace_bytes(P, G), ws)
    if not args.no_cpu_baseline:
        row_ptr, col = rp_d.cpu().numpy(), col_d.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(row_ptr, col, T, target_s=args.cpu_seconds)
        del row_ptr, col
    del ws
    torch.cuda.empty_cache()
    if args.packed_compare > 0 and not packed:
        out["packed_vs_plain"] = packed_leg(P, G, k, args, X0, elapsed / args.steps / B * 1e3)
    del G, rp_d, col_d
    torch.cuda.empty_cache()
    if not args.no_batched:
        print("[bench] plain vs batched", file=sys.stderr, flush=True)
        out["batched"] = batched_vs_plain(args)
        torch.cuda.empty_cache()
    if not args.no_serving:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serving_leg(args)
        out["p50_latency_s"] = out["serving"]["p50_latency_s"]
        out["p99_latency_s"] = out["serving"]["p99_latency_s"]
    return out


def beyond_hbm(args):
    """One colouring of a workload whose plain count does not fit in HBM, counted within
    --budget-gb of device workspace (cc_count_budget), twice at two budgets: the counts must agree
    (bit for bit when the budgets park the same tables and project alike, else within 1e-12)."""
    import torch

    import inputs
    import paper_1804_09764_amd as cc
    W = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    t0 = time.time()
    rp_d, col_d = inputs.rmat_graph_gpu(W["scale"], W["ef"], W["gseed"], device=dev)
    G = cc.Graph(rp_d, col_d, trust=W["trust"])
    P = cc.Plan(inputs.pruefer_tree(W["k"], W["tseed"]))
    print(f"[bench] graph n={G.n} nnz={G.nnz} in {time.time() - t0:.1f}s; plain workspace "
          f"{cc.count_workspace_bytes(P, G) / 1e9:.1f} GB, free {torch.cuda.mem_get_info(dev)[0] / 1e9:.1f} GB",
          file=sys.stderr, flush=True)
    C = cc.colour(G, W["k"], seed=args.seed, first_iter=0, B=1)
    out = {"workload": args.workload, "n": G.n, "nnz": G.nnz,
           "plain_workspace_GB": cc.count_workspace_bytes(P, G) / 1e9, "runs": []}
    ws = cc.Workspace()
    Xs = []
    budgets = (args.budget_gb, args.budget_gb * 0.85)
    infos = [cc.count_budget_plan(P, G, int(gb * 1e9)) for gb in budgets]
    # one host buffer for both runs (the larger need): page-locked if the host allows it, else
    # pageable (the copies are then staged by the runtime)
    hbytes = max(max(i["host_bytes"] for i in infos), 1)
    try:
        host = torch.empty(hbytes, dtype=torch.uint8, pin_memory=True)
        out["host_buffer"] = "page-locked"
    except Exception:
        host = torch.empty(hbytes, dtype=torch.uint8)
        out["host_buffer"] = "pageable"
    for gb, info in zip(budgets, infos):
        X = torch.empty(1, dtype=torch.float64, device=dev)
        cc.count_budget(P, G, C, int(gb * 1e9), workspace=ws, host=host, out=X)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cc.count_budget(P, G, C, int(gb * 1e9), workspace=ws, host=host, out=X)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3
        Xs.append(float(X.cpu()[0]))
        out["runs"].append({"budget_GB": gb, "workspace_GB": info["workspace_bytes"] / 1e9,
                            "host_GB": info["host_bytes"] / 1e9, "parked_tables": info["parked_tables"],
                            "proj_classes": info["proj_classes"], "arena_columns": info["arena_columns"],
                            "unbounded_columns": info["unbounded_columns"], "ms": ms, "X": Xs[-1],
                            "CSEU_per_s": float(G.nnz) * P.info.units_per_edge / (ms * 1e-3)})
        print(f"[bench] budget {gb:.0f} GB: {out['runs'][-1]}", file=sys.stderr, flush=True)
    out["agree"] = bool(Xs[0] == Xs[1] or abs(Xs[0] - Xs[1]) <= 1e-12 * max(Xs))
    return out


def packed_compare(args):
    """Packed against plain on a workload's own graph and template: the largest number of
    colourings (up to the workload's colourings per step) whose packed count fits in 85 % of the
    free HBM, counted once packed (one cc_count_packed) and once plain (one cc_count of the same
    colourings), after a warm-up of each. Reports time per colouring and whether the counts agree
    (exact below 2^53, 1e-12 relative above). Answers whether packing the colourings of the
    headline step would pay, with or without a device budget."""
    import numpy as np
    import torch

    import inputs
    import paper_1804_09764_amd as cc
    W = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    rp_d, col_d = inputs.rmat_graph_gpu(W["scale"], W["ef"], W["gseed"], device=dev)
    G = cc.Graph(rp_d, col_d, trust=W["trust"])
    P = cc.Plan(inputs.pruefer_tree(W["k"], W["tseed"]))
    free = torch.cuda.mem_get_info(dev)[0]
    need = {b: cc.count_packed_workspace_bytes(P, G, b) for b in range(1, W["B"] + 1)}
    fits = [b for b in need if need[b] <= 0.85 * free]
    out = {"workload": args.workload, "n": G.n, "nnz": G.nnz, "colourings_per_step": W["B"],
           "packed_workspace_GB": {str(b): need[b] / 1e9 for b in need},
           "plain_workspace_GB": cc.count_workspace_bytes(P, G) / 1e9, "free_GB": free / 1e9}
    if not fits:
        out["fits"] = False
        return out
    B = max(fits)
    C = cc.colour(G, W["k"], seed=args.seed, first_iter=0, B=B)
    Xp = torch.empty(B, dtype=torch.float64, device=dev)
    Xq = torch.empty(B, dtype=torch.float64, device=dev)
    res = {}
    for name, fn in (("plain", lambda ws: cc.count(P, G, C, workspace=ws, out=Xp)),
                     ("packed", lambda ws: cc.count_packed(P, G, C, workspace=ws, out=Xq))):
        ws = cc.Workspace()
        fn(ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(ws)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) * 1e3 / B
        print(f"[bench] {name}: {res[name]:.1f} ms per colouring ({B} colourings)", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    xp, xq = Xp.cpu().numpy(), Xq.cpu().numpy()
    small = xp < 2.0 ** 53
    agree = bool(np.array_equal(xp[small], xq[small]) and np.all(np.abs(xq - xp)[~small] <= 1e-12 * xp[~small]))
    out.update({"fits": True, "colourings": B, "plain_ms_per_colouring": res["plain"],
                "packed_ms_per_colouring": res["packed"], "packed_over_plain": res["packed"] / res["plain"],
                "agree": agree})
    return out


def packed_leg(P, G, k, args, X0, plain_ms):
    """The step's first colourings counted packed (as many as fit in 85 % of the free HBM, at most
    --packed-compare) against the plain count: its time per colouring in the timed steps, and its
    values for the same colourings (the first warm-up step; exact below 2^53, 1e-12 relative
    above). Reports whether packing the step's colourings would pay on this workload."""
    import numpy as np
    import torch

    import paper_1804_09764_amd as cc
    dev = torch.device("cuda:0")
    free = torch.cuda.mem_get_info(dev)[0]
    b = args.packed_compare
    while b > 0 and cc.count_packed_workspace_bytes(P, G, b) > 0.85 * free:
        b -= 1
    if b == 0:
        return {"fits": False, "plain_ms_per_colouring": plain_ms}
    C = cc.colour(G, k, seed=args.seed, first_iter=0, B=b)
    ws = cc.Workspace()
    Xq = torch.empty(b, dtype=torch.float64, device=dev)
    cc.count_packed(P, G, C, workspace=ws, out=Xq)  # warm-up (and the workspace's allocation)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cc.count_packed(P, G, C, workspace=ws, out=Xq)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / b
    agree = None
    if X0 is not None:
        xq, xp = Xq.cpu().numpy(), X0[:b].cpu().numpy()
        small = xp < 2.0 ** 53
        agree = bool(np.array_equal(xq[small], xp[small]) and np.all(np.abs(xq - xp)[~small] <= 1e-12 * xp[~small]))
    del ws
    torch.cuda.empty_cache()
    print(f"[bench] packed: {ms:.1f} ms per colouring ({b} colourings) against plain {plain_ms:.1f} ms",
          file=sys.stderr, flush=True)
    return {"fits": True, "colourings": b, "packed_ms_per_colouring": ms, "plain_ms_per_colouring": plain_ms,
            "packed_over_plain": ms / plain_ms, "agree_with_plain": agree,
            "packed_workspace_GB": cc.count_packed_workspace_bytes(P, G, b) / 1e9}


def budget_leg(P, G, k, args, full_bytes, ws):
    """One colouring of the headline workload counted within a device budget of budget_frac of the
    plain count's workspace (cc_count_budget: tables idle across the peak wait in pinned host
    memory), against the plain count of the same colouring: time, arenas, bytes parked, and
    whether the counts are bit-identical."""
    import torch

    import paper_1804_09764_amd as cc
    dev = torch.device("cuda:0")
    budget = int(full_bytes * args.budget_frac)
    try:
        info = cc.count_budget_plan(P, G, budget)
    except cc.CCError as e:
        return {"budget_GB": budget / 1e9, "fits": False, "error": str(e)}
    C = cc.colour(G, k, seed=args.seed, first_iter=10 ** 6, B=1)
    host = torch.empty(max(info["host_bytes"], 1), dtype=torch.uint8, pin_memory=True)
    X0 = torch.empty(1, dtype=torch.float64, device=dev)
    X1 = torch.empty(1, dtype=torch.float64, device=dev)
    res = {}
    for name, fn in (("plain", lambda: cc.count(P, G, C, workspace=ws, out=X0)),
                     ("budget", lambda: cc.count_budget(P, G, C, budget, workspace=ws, host=host, out=X1))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) * 1e3
    return {"budget_GB": budget / 1e9, "fits": True, "workspace_GB": info["workspace_bytes"] / 1e9,
            "plain_workspace_GB": full_bytes / 1e9, "parked_tables": info["parked_tables"],
            "host_GB": info["host_bytes"] / 1e9, "arena_columns": info["arena_columns"],
            "unbounded_columns": info["unbounded_columns"], "plain_ms": res["plain"], "budget_ms": res["budget"],
            "bit_identical": bool(torch.equal(X0, X1))}


def batched_vs_plain(args, reps: int = 2, inst_reps: int = 1):
    """Plain vs batched on the batched configuration: R-MAT scale 18 (edge factor 16, seed 2), all
    11 trees with 7 vertices x 64 colourings.

    plain   = one cc_count call per tree: colourings and splits one after another, one table row
              per (vertex, colouring);
    batched = one cc_count_packed_multi call: the 11 trees over the 64 colourings, every table row
              holding all 64 colourings, and the table of each distinct rooted sub-template
              computed once for all trees (exact below 2^53, 1e-12 relative above, against plain);
    packed_per_tree = one cc_count_packed call per tree (no sharing across trees);
    instances_persistent / instances_levels (with --instances) = the 704 (tree, colouring)
              instances in one persistent launch / one launch per dependency level (bit-identical
              to plain).
    All legs are credited with the same units: the trees' reference-partition units x 64."""
    import numpy as np
    import torch

    import inputs
    import paper_1804_09764_amd as cc

    from paper_1804_09764_amd import autotune

    dev = torch.device("cuda:0")
    rp_d, col_d = inputs.rmat_graph_gpu(18, 16, 2, device=dev)
    n, nnz = rp_d.numel() - 1, col_d.numel()
    G = cc.Graph(rp_d, col_d)
    trees = inputs.all_trees(7)
    plans = [cc.Plan(T) for T in trees]
    B = 64
    C = cc.colour(G, 7, seed=args.seed, first_iter=0, B=B)
    # the batched path's degree split and tile row, chosen by measurement before timing
    t0 = time.perf_counter()
    rec = autotune.tune_multi(plans, rp_d, col_d, B=B, seed=args.seed, repeats=2, trust=True)
    tune_s = time.perf_counter() - t0
    Gt = cc.Graph(rp_d, col_d, hub_threshold=rec.hub_threshold, chunk=rec.chunk, packed_tile=rec.packed_tile,
                  trust=True)
    print(f"[bench] batched autotune ({tune_s:.1f} s): tau={rec.hub_threshold} c={rec.chunk} "
          f"tile={rec.packed_tile} {rec.ms:.1f} ms (default {rec.default_ms:.1f} ms)", file=sys.stderr, flush=True)
    units = float(nnz) * sum(p.info.units_per_edge for p in plans) * B
    ws = cc.Workspace()
    Xp = torch.empty((len(plans), B), dtype=torch.float64, device=dev)

    def plain():
        for t, P in enumerate(plans):
            cc.count(P, G, C, workspace=ws, out=Xp[t])

    Xk = torch.empty((len(plans), B), dtype=torch.float64, device=dev)
    wsk = cc.Workspace()

    def packed():
        for t, P in enumerate(plans):
            cc.count_packed(P, Gt, C, workspace=wsk, out=Xk[t])

    multi = cc.Multi(plans)
    Xm = torch.empty((len(plans), B), dtype=torch.float64, device=dev)
    wsm = cc.Workspace()

    def shared():
        multi.count(Gt, C, workspace=wsm, out=Xm)

    Xq = torch.empty((len(plans), B), dtype=torch.float64, device=dev)
    wsq = cc.Workspace()

    def persistent_multi():
        multi.count(Gt, C, workspace=wsq, out=Xq, persistent=True)

    legs = [("plain", plain), ("batched", shared)]
    if not args.no_persistent:
        legs.append(("batched_persistent", persistent_multi))
    legs.append(("packed_per_tree", packed))
    Xb = torch.empty((len(plans), B), dtype=torch.float64, device=dev)
    inst = [(P, G, C[b], Xb[t, b:b + 1], None) for t, P in enumerate(plans) for b in range(B)]
    if args.instances:
        persistent = cc.Batch(inst)
        levels = cc.Batch(inst, levels=True)
        wsb = cc.Workspace()
        legs += [("instances_persistent", lambda: persistent.run(wsb)), ("instances_levels", lambda: levels.run(wsb))]
    res = {}
    for name, fn in legs:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = inst_reps if name.startswith("instances") else reps
        for _ in range(r):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / r
        print(f"[bench] {name}: {res[name] * 1e3:.1f} ms", file=sys.stderr, flush=True)
        if name == "instances_persistent":
            persistent.check()
        if name.startswith("instances"):
            res[name + "_equal"] = bool(torch.equal(Xb, Xp))
    xp = Xp.cpu().numpy()
    small = xp < 2.0 ** 53

    def matches(x):
        return bool(np.array_equal(x[small], xp[small]) and
                    (np.all(np.abs(x[~small] - xp[~small]) <= 1e-12 * xp[~small]) if (~small).any() else True))
    out = {"workload": "rmat18-ef16-trees7x64",
            "graph": "R-MAT scale 18 edge factor 16 seed 2", "n": n, "nnz": nnz,
            "templates": "all 11 trees with 7 vertices", "colourings": B, "instances": len(inst),
            "units": units,
            "plain": {"value": units / res["plain"], "ms": res["plain"] * 1e3},
            "batched": {"value": units / res["batched"], "ms": res["batched"] * 1e3,
                        "speedup_vs_plain": res["plain"] / res["batched"],
                        "matches_plain": matches(Xm.cpu().numpy()), "above_2_53": int((~small).sum()),
                        "launch": "one packed multi-template count, one launch per split: 64 colourings per "
                                  "table row, equal sub-template tables shared by the 11 trees",
                        "splits_run": multi.info["steps"], "splits_total": multi.info["splits"],
                        "autotuned": {"hub_threshold": rec.hub_threshold, "chunk": rec.chunk,
                                      "packed_tile": rec.packed_tile, "ms": rec.ms, "default_ms": rec.default_ms,
                                      "candidates": len(rec.timings), "tuning_s": tune_s}},
            "packed_per_tree": {"value": units / res["packed_per_tree"], "ms": res["packed_per_tree"] * 1e3,
                                "matches_plain": matches(Xk.cpu().numpy()),
                                "launch": "one packed count per tree"},
            "workspace_GB": {"batched": multi.workspace_bytes(G, B) / 1e9,
                             "batched_persistent": multi.workspace_bytes(G, B, persistent=True) / 1e9,
                             "packed_per_tree": max(cc.count_packed_workspace_bytes(p, G, B) for p in plans) / 1e9}}
    if not args.no_persistent:
        out["batched_persistent"] = {"value": units / res["batched_persistent"], "ms": res["batched_persistent"] * 1e3,
                                     "speedup_vs_plain": res["plain"] / res["batched_persistent"],
                                     "equal_to_batched": bool(torch.equal(Xq, Xm)),
                                     "launch": "the same count in one persistent cooperative launch over (split, "
                                               "task or cut row, colouring tile) items, dependency levels separated "
                                               "by a device-wide barrier"}
    if args.instances:
        out["instances_persistent"] = {"value": units / res["instances_persistent"],
                                       "ms": res["instances_persistent"] * 1e3,
                                       "equal_to_plain": res["instances_persistent_equal"],
                                       "launch": "704 instances, one persistent launch"}
        out["instances_levels"] = {"value": units / res["instances_levels"], "ms": res["instances_levels"] * 1e3,
                                   "equal_to_plain": res["instances_levels_equal"],
                                   "launch": "704 instances, one launch per dependency level"}
        out["workspace_GB"]["instances"] = persistent.workspace_bytes / 1e9
    return out


SERVE_POOL = [(16 + (i % 7), (8, 16, 32)[i % 3], 100 + i) for i in range(16)]  # (scale, edge factor, seed)
# request mixes: "full" draws every graph of the pool and 8..128 colourings per request; "light"
# keeps k in 5..12 but draws only the graphs of scale <= 20 and 8..16 colourings, so that 100 or
# more requests per arrival rate fit in the benchmark's time; "bench" is "light" with one request
# in ten a large one of 64..128 colourings (the head-of-line case)
SERVE_MIXES = {"full": dict(max_scale=22, b_range=(8, 128), large=0.0),
               "light": dict(max_scale=20, b_range=(8, 16), large=0.0),
               "bench": dict(max_scale=20, b_range=(8, 16), large=0.1)}
LARGE_B = (64, 128)  # colourings of the occasional large request of the "bench" mix


def make_requests(n, pool, seed, rate, k_range=(5, 12), b_range=(8, 128), max_scale=22, large=0.0, t0=0.0):
    """n requests with Poisson arrivals at `rate` per second (all at t0 if rate is 0): a graph
    uniform over the pool's graphs of scale <= max_scale, a Pruefer tree with k uniform in k_range
    (seeded by the request id), B uniform in b_range colourings, or with probability `large` in
    LARGE_B. The same seed gives the same requests whatever the rate."""
    import numpy as np

    import inputs
    from paper_1804_09764_amd.serving import Request
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng(seed + 1)
    gids = [i for i, (scale, _, _) in enumerate(pool) if scale <= max_scale]
    t = t0
    out = []
    for i in range(n):
        if rate > 0:
            t += arr.exponential(1.0 / rate)
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        B = int(rng.integers(b_range[0], b_range[1] + 1))
        if rng.random() < large:
            B = int(rng.integers(LARGE_B[0], LARGE_B[1] + 1))
        gid = gids[int(rng.integers(0, len(gids)))]
        rid = seed * 100000 + i
        out.append(Request(rid=rid, graph_id=gid, tree_edges=inputs.pruefer_tree(k, rid), B=B, seed=rid, arrival=t))
    return out


def serving_leg(args):
    """Continuous-batching server over 16 resident R-MAT graphs (scale 16..22, edge factor 8..32).

    One request mix (seed 9) throughout: first the capacity, with all of its requests queued at
    once; then the same requests with Poisson arrivals at fractions of that capacity (--serve-loads,
    80 % and 95 % by default).
    Reports served CSEU/s and p50/p99 latency (arrival to result) per load, with each request's
    colourings capped per batch (slot_colourings) so that small requests share the batches of large
    ones; at the highest load the same arrivals also run first come, first served without the cap,
    which shows the head-of-line blocking the cap relieves (latencies of the smaller and larger
    halves of the requests reported apart). The 80 % figures are the headline latencies."""
    import numpy as np
    import torch

    import inputs
    import paper_1804_09764_amd as cc
    from paper_1804_09764_amd.serving import GpuExecutor, Server, latency_summary

    dev = torch.device("cuda:0")
    mix = SERVE_MIXES[args.serve_mix]
    pool, pool_desc = [], []
    for scale, ef, seed in SERVE_POOL:
        rp, col = inputs.rmat_graph_gpu(scale, ef, seed, device=dev)
        pool.append(cc.Graph(rp, col, trust=True))
        pool_desc.append((scale, ef, seed))
    units_cache = {}

    def units(r):
        key = r.tree_edges.tobytes()
        if key not in units_cache:
            units_cache[key] = cc.Plan(r.tree_edges, bind=False).info.units_per_edge
        return float(pool[r.graph_id].nnz) * units_cache[key] * r.B

    ex = GpuExecutor(pool, seed_base=args.seed, n_streams=2)
    budget = int(args.serve_budget_gb * 1e9)
    nreq = args.serve_requests

    def reqs_at(rate):
        return make_requests(nreq, pool_desc, seed=9, rate=rate, b_range=mix["b_range"], max_scale=mix["max_scale"],
                             large=mix["large"])

    def progress(r):
        if r.rid % 20 == 19:
            print(f"[bench] served request {r.rid}: k={r.k} B={r.B} {r.status} latency {r.latency:.2f}s",
                  file=sys.stderr, flush=True)

    def serve(reqs, cap):
        srv = Server(ex, budget, max_inflight=2, slot_colourings=cap, on_complete=progress)
        t0 = time.perf_counter()
        srv.run(reqs)
        return srv, time.perf_counter() - t0

    def summary(reqs, srv, wall, rate):
        lat = latency_summary(reqs)
        served = sum(units(r) for r in reqs if r.status == "done")
        work = np.array([units(r) for r in reqs])
        small = work <= np.median(work)
        ls = latency_summary([r for r, m in zip(reqs, small) if m])
        lb = latency_summary([r for r, m in zip(reqs, small) if not m])
        return {"arrival_rate_per_s": rate, "requests": len(reqs), "failed": sum(r.status != "done" for r in reqs),
                "wall_s": wall, "throughput_CSEU_per_s": served / wall,
                "p50_latency_s": lat.get("p50_s"), "p99_latency_s": lat.get("p99_s"), "mean_latency_s": lat.get("mean_s"),
                "smaller_half_p50_s": ls.get("p50_s"), "smaller_half_p99_s": ls.get("p99_s"),
                "larger_half_p50_s": lb.get("p50_s"), "larger_half_p99_s": lb.get("p99_s"),
                "batches": srv.stats.batches,
                "mean_colourings_per_batch": (sum(srv.stats.batch_sizes) / max(1, srv.stats.batches)),
                "max_inflight_batches": srv.stats.max_inflight_batches,
                "max_inflight_GB": srv.stats.max_inflight_bytes / 1e9}

    # warm up (plans, allocator) on a few small requests
    warm = make_requests(4, pool_desc, seed=1, rate=0, b_range=(2, 4), max_scale=18)
    Server(ex, budget, max_inflight=2).run(warm)
    torch.cuda.synchronize()
    cap_reqs = reqs_at(0)
    srv, makespan = serve(cap_reqs, args.serve_cap)
    capacity = len(cap_reqs) / makespan
    cap_units = sum(units(r) for r in cap_reqs if r.status == "done")
    print(f"[bench] serving capacity {capacity:.3f} requests/s ({makespan:.1f} s for {len(cap_reqs)})",
          file=sys.stderr, flush=True)
    loads = {}
    for load in args.serve_loads:
        rate = load * capacity
        reqs = reqs_at(rate)
        srv, wall = serve(reqs, args.serve_cap)
        loads[f"{load:.2f}"] = summary(reqs, srv, wall, rate)
        print(f"[bench] Poisson arrivals at {load:.2f} x capacity = {rate:.3f}/s: {wall:.1f} s, "
              f"p50 {loads[f'{load:.2f}']['p50_latency_s']:.2f} s p99 {loads[f'{load:.2f}']['p99_latency_s']:.2f} s",
              file=sys.stderr, flush=True)
    fifo = None
    if args.serve_fifo_load > 0:
        rate = args.serve_fifo_load * capacity
        reqs = reqs_at(rate)
        srv, wall = serve(reqs, 0)
        fifo = summary(reqs, srv, wall, rate)
        fifo["load"] = args.serve_fifo_load
        print(f"[bench] first come first served, no cap, at {args.serve_fifo_load:.2f} x capacity: "
              f"p50 {fifo['p50_latency_s']:.2f} s p99 {fifo['p99_latency_s']:.2f} s", file=sys.stderr, flush=True)
    head = loads.get("0.80") or next(iter(loads.values()))
    return {"workload": f"Poisson requests over 16 resident R-MAT graphs (scale 16-22, edge factor 8-32), "
                        f"Pruefer trees k in 5..12; mix '{args.serve_mix}': graphs of scale <= {mix['max_scale']}, "
                        f"{mix['b_range'][0]}..{mix['b_range'][1]} colourings per request"
                        + (f", one request in {round(1 / mix['large'])} with {LARGE_B[0]}..{LARGE_B[1]}"
                           if mix["large"] > 0 else "")
                        + f"; the same {nreq} requests (seed 9) for the capacity and every load",
            "slot_colourings": args.serve_cap,
            "capacity_requests_per_s": capacity, "capacity_CSEU_per_s": cap_units / makespan,
            "memory_budget_GB": budget / 1e9, "loads": loads, "fifo_uncapped": fifo,
            "p50_latency_s": head["p50_latency_s"], "p99_latency_s": head["p99_latency_s"],
            "throughput_CSEU_per_s": head["throughput_CSEU_per_s"]}


COUNT_KERNELS = ("k_edge_colours", "k_project", "k_split", "k_hub_finish", "k_reduce_blocks", "k_reduce_final")


def dispatch_sequence(P, G, proj):
    """The kernels cc_count dispatches for one colouring, in order, each with the split it belongs
    to (-1: none): the neighbour-colour gather; per split either its task kernel or, when projected,
    a copy and a task kernel per pass of colour classes, then the cut-row finish; the root sum."""
    seq = [("k_edge_colours", -1)]
    tasks = G.info["n_chunks"] + G.info["n_light"] > 0
    for i in range(P.info.n_splits):
        if proj[i] > 0:
            passes = -(-P.k // proj[i])
            per = -(-P.k // passes)
            for c0 in range(0, P.k, per):
                seq.append(("k_project", i))
                if tasks:
                    seq.append(("k_split", i))
        elif tasks:
            seq.append(("k_split", i))
        if G.info["n_hubs"] > 0:
            seq.append(("k_hub_finish", i))
    seq += [("k_reduce_blocks", -1), ("k_reduce_final", -1)]
    return seq


def summarize_pmc(args):
    """rocprofv3 --pmc output (counter_collection.csv of a FETCH_SIZE run and of a WRITE_SIZE run)
    -> pmc_<workload>.json (or --out): the bytes one colouring's dominant split moves (all of its
    kernels: row copies, passes, cut-row finish), scaled by what the same counters read for a plain
    copy of known size. Dispatches are matched to splits by cc_count's launch sequence
    (dispatch_sequence, written by the profiled bench run with --dispatch-map)."""
    def rows(d):
        out = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                out += list(csv.DictReader(fh))
        return out

    def dispatches(rs, counter):
        out = []
        for r in sorted(rs, key=lambda r: int(r.get("Dispatch_Id", 0))):
            if r.get("Counter_Name") == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out

    dm = json.load(open(args.dispatch_map))
    seq = [tuple(x) for x in dm["sequence"]]
    dom = dm["dominant_split"]

    def per_colouring(ds):
        copy = [v for name, v in ds if "copybuffer" in name.lower()]
        ours = [(name, v) for name, v in ds if any(k in name for k in COUNT_KERNELS)]
        if len(ours) % len(seq):
            raise SystemExit(f"{len(ours)} count dispatches are not a whole number of {len(seq)}-kernel colourings")
        per = []
        for c0 in range(0, len(ours), len(seq)):
            total = 0.0
            for (name, v), (kname, split) in zip(ours[c0:c0 + len(seq)], seq):
                if kname not in name:
                    raise SystemExit(f"dispatch {name} where {kname} was expected")
                if split == dom:
                    total += v
            per.append(total)
        return per, (sorted(copy[:3])[1] if len(copy) >= 3 else None)

    fper, fk = per_colouring(dispatches(rows(args.fetch_dir), "FETCH_SIZE"))
    wper, wk = per_colouring(dispatches(rows(args.write_dir), "WRITE_SIZE"))
    f_factor = args.copy_bytes / (fk * 1024.0) if fk else 1.0
    w_factor = args.copy_bytes / (wk * 1024.0) if wk else 1.0
    fetch_kib = sum(fper) / len(fper)
    write_kib = sum(wper) / len(wper)
    res = {"workload": args.workload, "kernel_hash": kernel_hash(args.workload), "split_index": dom,
           "kernels": sorted({k for k, s_ in seq if s_ == dom}), "colourings": len(fper),
           "fetch_kib_per_colouring": fetch_kib, "write_kib_per_colouring": write_kib,
           "copy_fetch_factor": f_factor, "copy_write_factor": w_factor,
           "traffic_bytes_per_launch": fetch_kib * 1024.0 * f_factor + write_kib * 1024.0 * w_factor,
           "command": args.command}
    path = args.out or f"pmc_{args.workload}.json"
    json.dump(res, open(path, "w"), indent=1)
    print(json.dumps(res))


def summarize_stats(args):
    """rocprofv3 --kernel-trace --stats output (kernel_stats.csv) -> a markdown table of the kernels'
    calls and durations, printed (copied into profiles/ with the command that made it)."""
    f = glob.glob(os.path.join(args.stats_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit("no kernel_stats.csv under " + args.stats_dir)
    rows = list(csv.DictReader(open(f[0])))
    agg = {}
    for r in rows:
        name = r["Name"].replace("(anonymous namespace)::", "")
        name = re.sub(r"\(.*", "", name).replace("void ", "").strip()[:60]
        name = re.sub(r"^.*::", "", name.split("<")[0]) + ("<" + name.split("<", 1)[1] if "<" in name else "")
        a = agg.setdefault(name, [0, 0.0])
        a[0] += int(r["Calls"])
        a[1] += float(r["TotalDurationNs"]) / 1e6
    total = sum(a[1] for a in agg.values())
    print(f"# rocprofv3 kernel summary: {args.title}\n")
    print("command (from the repository root on the MI355X box):\n  " + args.command + "\n")
    print(f"bench.py kernel_hash of the split kernel's code and this template's plan constants: "
          f"{kernel_hash(args.workload)}\n")
    print("| kernel | calls | total ms | average ms | % |\n|---|---|---|---|---|")
    for name, (calls, ms) in sorted(agg.items(), key=lambda x: -x[1][1]):
        if ms < 0.01:
            continue
        print(f"| {name} | {calls} | {ms:.2f} | {ms / calls:.3f} | {100 * ms / total:.2f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=777)
    ap.add_argument("--hub-threshold", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--autotune", default="", metavar="CACHE.json",
                    help="pick the hub threshold and chunk size by timing candidates first (records "
                         "cached in this JSON file)")
    ap.add_argument("--path", default="auto", choices=("auto", "packed", "plain"),
                    help="packed: the colourings of a step share the table rows (cc_count_packed); "
                         "plain: one colouring after another (cc_count); auto: packed when the step has "
                         "at least 8 colourings and they fit in one packed count, else plain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the plain-vs-batched comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the plain-vs-batched comparison (for profiling its kernels)")
    ap.add_argument("--progress", type=int, default=1,
                    help="print a line after each timed step (synchronises between steps)")
    ap.add_argument("--serve-requests", type=int, default=100,
                    help="requests of the capacity run and of each arrival rate (the same requests)")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.8, 0.95],
                    help="Poisson arrival rates as fractions of the measured capacity")
    ap.add_argument("--serve-mix", default="light", choices=sorted(SERVE_MIXES))
    ap.add_argument("--serve-cap", type=int, default=4,
                    help="colourings of one request per batch (0: as many as fit)")
    ap.add_argument("--serve-fifo-load", type=float, default=0.95,
                    help="also run this load without the cap, first come first served (0: skip)")
    ap.add_argument("--only-serving", action="store_true", help="run only the serving leg")
    ap.add_argument("--only-budget", action="store_true",
                    help="count one colouring of --workload within --budget-gb of device workspace")
    ap.add_argument("--budget-gb", type=float, default=290.0)
    ap.add_argument("--serve-budget-gb", type=float, default=160.0)
    ap.add_argument("--cpu-seconds", type=float, default=6.0)
    ap.add_argument("--no-persistent", action="store_true",
                    help="skip the batched leg's persistent (cooperative) launch, e.g. under a kernel trace")
    ap.add_argument("--instances", action="store_true",
                    help="also time the instance batches (704 instances in one or a few launches)")
    ap.add_argument("--packed-compare", type=int, default=2,
                    help="also count this many of the step's colourings packed (fewer if they do not fit; "
                         "0: skip) and compare with the plain count")
    ap.add_argument("--only-packed-compare", action="store_true",
                    help="packed counts of the largest colouring batch that fits against plain counts "
                         "of the same colourings, on --workload")
    ap.add_argument("--budget-frac", type=float, default=0.9,
                    help="also count one colouring within this fraction of the plain workspace (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--summarize-pmc", action="store_true")
    ap.add_argument("--fetch-dir")
    ap.add_argument("--write-dir")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--dispatch-map", default="",
                    help="write (bench run) or read (--summarize-pmc) the count's kernel sequence per colouring")
    ap.add_argument("--out", default="")
    ap.add_argument("--summarize-stats", default="", metavar="DIR")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", default="")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args)
        return 0
    if args.summarize_stats:
        args.stats_dir = args.summarize_stats
        summarize_stats(args)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the counting path does not span GPUs "
              "(it would shard by colouring, or by colour-set column for a colouring too large "
              "for one GPU; neither is built).",
              file=sys.stderr)
        return 2
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only_budget:
        print(json.dumps({"beyond_hbm": beyond_hbm(args)}), flush=True)
        return 0
    if args.only_serving:
        print(json.dumps({"serving": serving_leg(args)}), flush=True)
        return 0
    if args.only_packed_compare:
        print(json.dumps({"packed_compare": packed_compare(args)}), flush=True)
        return 0
    if args.only_batched:
        # the batched leg alone (for profiling its kernels); not the benchmark line
        print(json.dumps({"batched": batched_vs_plain(args)}), flush=True)
        return 0
    out = bench(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
